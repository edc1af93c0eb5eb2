// Krylov stage solve (App. A eq. linsystem_primal, and eq. linsystem_adjoint
// for the adjoint): the fallback for the steps whose splitting iteration
// would not contract (bound theta >= 0.5).  The paper solves every stage
// system with GMRES; here restarted GMRES runs only on those steps.
//
// The operator is block diagonal over the streamed batch: entry e of
// segment s belongs to system s, so (A x)_e = x_e - h_s (M_s x)_e with the
// step's controls, and the Krylov vectors span the whole batch.  Right
// preconditioning by the diagonal W = (1 - h D)^{-1} (the weight of the
// splitting iteration) gives B y = A (W y); the solution is z = W y.  These
// kernels are the vector operations of that iteration; the Arnoldi loop and
// the small least-squares problem run on the host.
#include <hip/hip_runtime.h>

#include "lbx_host.hpp"

namespace lbx {

namespace {

__device__ __forceinline__ int kry_seg(const StreamSeg *segs, int nseg, int64_t blk) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Entry of this thread: segment, system, index within the state and the
// diagonal data; false past the segment's end.
struct KryEntry {
  int64_t e, r, base;
  uint64_t di, dj;
  double gam, dE;
};

__device__ __forceinline__ bool kry_entry(const KryArgs &A, const SysDev *&Sp, KryEntry &k) {
  const int64_t u = blockIdx.x;
  const StreamSeg &sg = A.segs[kry_seg(A.segs, A.nseg, u)];
  const SysDev &S = A.sysv[sg.sys];
  Sp = &S;
  const int64_t local = (u - sg.blk0) * STREAM_BLOCK + threadIdx.x;
  if (local >= sg.count) return false;
  const int64_t b = local / S.N2;
  k.r = local - b * S.N2;
  const int i = (int)(k.r / S.N);
  const int jj = (int)(k.r - (int64_t)i * S.N);
  k.di = A.desc[S.tab_off + i];
  k.dj = A.desc[S.tab_off + jj];
  k.gam = diag_rate(S, k.di, k.dj);
  k.dE = A.Etab[S.tab_off + i] - A.Etab[S.tab_off + jj];
  k.base = sg.off + b * S.N2;
  k.e = k.base + k.r;
  return true;
}

// u = W x.
template <bool ADJ>
__global__ __launch_bounds__(STREAM_BLOCK) void kry_weight_kernel(KryArgs A, const double2 *__restrict__ x,
                                                                  double2 *__restrict__ u) {
  const SysDev *S;
  KryEntry k;
  if (!kry_entry(A, S, k)) return;
  u[k.e] = cmul(stage_weight(S->h, k.gam, k.dE, ADJ), x[k.e]);
}

// y = A u, or y = q - A u when q is not NULL.
template <bool ADJ>
__global__ __launch_bounds__(STREAM_BLOCK) void kry_apply_kernel(KryArgs A, const double2 *__restrict__ u,
                                                                 const double2 *__restrict__ q,
                                                                 double2 *__restrict__ y) {
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dq[QMAX];
  __shared__ double2 jq[JCMAX];
  const int tid = threadIdx.x;
  const StreamSeg &sg0 = A.segs[kry_seg(A.segs, A.nseg, blockIdx.x)];
  const SysDev &S0 = A.sysv[sg0.sys];
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  if (tid < S0.Q) dq[tid] = A.ctab[S0.ctab_off + (int64_t)A.j * S0.Q + tid];
  if (tid < S0.njc) jq[tid] = jc_coef(S0, tid, ((double)A.j + 0.5) * S0.dt);
  __syncthreads();
  const SysDev *S;
  KryEntry k;
  if (!kry_entry(A, S, k)) return;
  const double2 *us = u + k.base;
  const double2 acc = offdiag_all<ADJ>(*S, k.di, k.dj, k.r, dq, jq, sq, [&](int64_t idx) { return us[idx]; });
  const double2 own = us[k.r];
  const double2 Mu = cadd(acc, cmul(diag_coef(k.gam, k.dE, ADJ), own));
  const double2 Au = csub(own, cscale(S->h, Mu));
  y[k.e] = q ? csub(q[k.e], Au) : Au;
}

// Partial inner products <V_i, x> (conjugate-linear in V_i), i < n, of the
// entries of this workgroup (grid-stride), one row of n per workgroup.
__global__ __launch_bounds__(256) void kry_dot_kernel(const double2 *__restrict__ V, int64_t stride, int n,
                                                      const double2 *__restrict__ x, int64_t E,
                                                      double2 *__restrict__ part) {
  __shared__ double red[2][KRY_MAXV][4];
  double2 acc[KRY_MAXV];
#pragma unroll
  for (int i = 0; i < KRY_MAXV; ++i) acc[i] = make_double2(0.0, 0.0);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < E; e += (int64_t)gridDim.x * 256) {
    const double2 xv = x[e];
#pragma unroll
    for (int i = 0; i < KRY_MAXV; ++i)
      if (i < n) {
        const double2 v = V[i * stride + e];
        acc[i].x += v.x * xv.x + v.y * xv.y;
        acc[i].y += v.x * xv.y - v.y * xv.x;
      }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < KRY_MAXV; ++i)
    if (i < n) {
      double re = acc[i].x, im = acc[i].y;
      for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_down(re, off, 64);
        im += __shfl_down(im, off, 64);
      }
      if (lane == 0) {
        red[0][i][wv] = re;
        red[1][i][wv] = im;
      }
    }
  __syncthreads();
  if (threadIdx.x < n) {
    const int i = threadIdx.x;
    part[(int64_t)blockIdx.x * KRY_MAXV + i] =
        make_double2(red[0][i][0] + red[0][i][1] + red[0][i][2] + red[0][i][3],
                     red[1][i][0] + red[1][i][1] + red[1][i][2] + red[1][i][3]);
  }
}

// out[i] = sum over the rows of part[.][i], one wavefront per i.
__global__ __launch_bounds__(64) void kry_reduce_kernel(const double2 *__restrict__ part, int rows, int n,
                                                        double2 *__restrict__ out) {
  const int i = blockIdx.x;
  if (i >= n) return;
  double re = 0.0, im = 0.0;
  for (int r = threadIdx.x; r < rows; r += 64) {
    const double2 v = part[(int64_t)r * KRY_MAXV + i];
    re += v.x;
    im += v.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    re += __shfl_down(re, off, 64);
    im += __shfl_down(im, off, 64);
  }
  if (threadIdx.x == 0) out[i] = make_double2(re, im);
}

// x = s x - sum_{i < n} c_i V_i.
__global__ __launch_bounds__(256) void kry_axpy_kernel(const double2 *__restrict__ V, int64_t stride, KryCoef c,
                                                       double s, double2 *__restrict__ x, int64_t E) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < E; e += (int64_t)gridDim.x * 256) {
    double2 v = cscale(s, x[e]);
#pragma unroll
    for (int i = 0; i < KRY_MAXV; ++i)
      if (i < c.n) v = csub(v, cmul(c.c[i], V[i * stride + e]));
    x[e] = v;
  }
}

// z = W y; out = 2 z - q (eq. IMR: q + dt M z = 2 z - q); zh = z when given.
template <bool ADJ>
__global__ __launch_bounds__(STREAM_BLOCK) void kry_finish_kernel(KryArgs A, const double2 *__restrict__ y,
                                                                  const double2 *__restrict__ q,
                                                                  double2 *__restrict__ out,
                                                                  double2 *__restrict__ zh) {
  const SysDev *S;
  KryEntry k;
  if (!kry_entry(A, S, k)) return;
  const double2 z = cmul(stage_weight(S->h, k.gam, k.dE, ADJ), y[k.e]);
  out[k.e] = csub(cscale(2.0, z), q[k.e]);
  if (zh) zh[k.e] = z;
}

unsigned vec_grid(int64_t E) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((E + 255) / 256, 1024)); }

}  // namespace

int launch_kry_weight(const KryArgs &A, bool adj, const double2 *x, double2 *u, hipStream_t st) {
  if (adj)
    hipLaunchKernelGGL(kry_weight_kernel<true>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, x, u);
  else
    hipLaunchKernelGGL(kry_weight_kernel<false>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, x, u);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

int launch_kry_apply(const KryArgs &A, bool adj, const double2 *u, const double2 *q, double2 *y, hipStream_t st) {
  if (adj)
    hipLaunchKernelGGL(kry_apply_kernel<true>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, u, q, y);
  else
    hipLaunchKernelGGL(kry_apply_kernel<false>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, u, q, y);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

size_t kry_part_bytes() { return (size_t)1024 * KRY_MAXV * sizeof(double2) + KRY_MAXV * sizeof(double2); }

int launch_kry_dots(const double2 *V, int64_t stride, int n, const double2 *x, int64_t E, double2 *part,
                    double2 *out, hipStream_t st) {
  if (n < 1 || n > KRY_MAXV) return fail(LB_EINVAL, "Krylov dot count out of range");
  const unsigned g = vec_grid(E);
  hipLaunchKernelGGL(kry_dot_kernel, dim3(g), dim3(256), 0, st, V, stride, n, x, E, part);
  LBX_HIP(hipGetLastError());
  hipLaunchKernelGGL(kry_reduce_kernel, dim3((unsigned)n), dim3(64), 0, st, part, (int)g, n, out);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

int launch_kry_axpy(const double2 *V, int64_t stride, const KryCoef &c, double s, double2 *x, int64_t E,
                    hipStream_t st) {
  if (c.n < 0 || c.n > KRY_MAXV) return fail(LB_EINVAL, "Krylov coefficient count out of range");
  hipLaunchKernelGGL(kry_axpy_kernel, dim3(vec_grid(E)), dim3(256), 0, st, V, stride, c, s, x, E);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

int launch_kry_finish(const KryArgs &A, bool adj, const double2 *y, const double2 *q, double2 *out, double2 *zh,
                      hipStream_t st) {
  if (adj)
    hipLaunchKernelGGL(kry_finish_kernel<true>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, y, q, out,
                       zh);
  else
    hipLaunchKernelGGL(kry_finish_kernel<false>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, y, q, out,
                       zh);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

}  // namespace lbx
