// Streaming kernels: control table, matrix-free apply of M(t), the adjoint
// gradient integrands, the adjoint terminal condition, objective reductions
// and the gradient contraction.  Every kernel reads and writes states in HBM
// (or cache).  The stage solves of streamed systems run in the persistent
// step kernels of kernels_step.hip; the LDS-resident persistent kernels for
// small systems live in kernels_lds.hip and kernels_lds_fast.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbx_host.hpp"

namespace lbx {

// Zeroes n 32-bit words (a kernel rather than hipMemsetAsync, so that a
// caller may capture the launches of a call in a graph).
__global__ void fill_zero_kernel(uint32_t *__restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// A deterministic, non-zero trial state for the autotuner: entry k gets
// 1e-2 (u, v) with u, v in [-1, 1) from a splitmix64 hash of k.  (Timing on
// zeros runs faster than on a real trajectory and can reorder the kernels.)
__device__ __forceinline__ double hash_unit(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void fill_trial_kernel(double2 *__restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(1e-2 * hash_unit(2 * (uint64_t)i), 1e-2 * hash_unit(2 * (uint64_t)i + 1));
}

int launch_fill_trial(double2 *ptr, int64_t n, hipStream_t st) {
  if (n == 0) return LB_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_trial_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ptr, n);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

int launch_fill_zero(void *ptr, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n == 0) return LB_OK;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint32_t *)ptr, n);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// ----------------------------------------------------------------------------
// Control table (Sec. II eq. rotctrl, evaluated at step midpoints, App. A)
// and the contraction bound of every step's stage solve.
//
// The stage system (I - h M) z = q, h = dt/2, M = D + O, is solved by the
// fixed-point iteration z <- w (q + h O z) with w = (1 - h D)^-1.  Since
// Re D <= 0, |w| <= 1 and the iteration contracts in the max norm with
// factor theta <= h max_row sum|O| <= h sum_q (2 |d_q| c_q + (n_q - 1)/T1_q).
// ttab receives (theta, theta / (1 - theta)) for the a-posteriori counts of
// the streamed step kernels and the specialised LDS kernels; ktab the
// a-priori counts of the generic LDS kernels (started from z0 = w q the
// error after K sweeps is <= theta^(K+1) |z|) and of a start from z0 = q
// (<= theta^K (h max|D| + theta) |z|), which sweep_counts reports.
// ----------------------------------------------------------------------------
__global__ void control_table_kernel(const SysDev *__restrict__ sysv, int s0, int NT,
                                     const double *__restrict__ alpha,
                                     const double *__restrict__ carrier, double2 *__restrict__ ctab,
                                     int64_t ctab_shift, int32_t *__restrict__ ktab,
                                     double2 *__restrict__ ttab, double tol) {
  const int s = s0 + (int)blockIdx.y;
  const SysDev &S = sysv[s];
  const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= NT) return;
  const double t = ((double)j + 0.5) * S.dt;
  double theta = S.theta_jump;
  for (int q = 0; q < S.Q; ++q) {
    const double2 d = control_value(S, alpha + S.alpha_off, carrier + S.carrier_off, q, t);
    ctab[S.ctab_off - ctab_shift + (int64_t)j * S.Q + q] = d;
    theta += S.h * 2.0 * hypot(d.x, d.y) * S.csum[q];
  }
  if (ttab) ttab[(int64_t)s * NT + j] = make_double2(theta, theta < 1.0 ? theta / (1.0 - theta) : 0.0);
  if (ktab) {
    int klds, kst;
    if (!(theta < 0.5)) {
      klds = kst = -1;
    } else if (theta <= 0.0) {
      klds = kst = 1;
    } else {
      const double lt = log(theta);
      const double ltol = log(tol);
      klds = (int)ceil(ltol / lt) - 1;
      klds = klds < 1 ? 1 : klds;
      const double e0 = S.hDmax + theta;
      kst = e0 <= tol ? 1 : (int)ceil((ltol - log(e0)) / lt);
      kst = kst < 1 ? 1 : kst;
    }
    ktab[((int64_t)s * NT + j) * 2 + 0] = klds;
    ktab[((int64_t)s * NT + j) * 2 + 1] = kst;
  }
}

int launch_control_table(const lb_plan *p, int s0, int nsys, const double *alpha, double2 *ctab,
                         int64_t ctab_shift, int32_t *ktab, double2 *ttab, double tol, hipStream_t st) {
  dim3 grid((p->NT + 255) / 256, nsys);
  hipLaunchKernelGGL(control_table_kernel, grid, dim3(256), 0, st, p->d_sys, s0, p->NT, alpha,
                     p->d_carrier, ctab, ctab_shift, ktab, ttab, tol);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// ----------------------------------------------------------------------------
// y = M(t) x or M(t)^+ x for B states of one system.
// ----------------------------------------------------------------------------
template <bool ADJ>
__global__ __launch_bounds__(STREAM_BLOCK) void apply_kernel(
    const SysDev *__restrict__ sysv, int sys, double t, const double *__restrict__ alpha,
    const double *__restrict__ carrier, const double *__restrict__ Etab,
    const uint64_t *__restrict__ desc, const double2 *__restrict__ x, double2 *__restrict__ y,
    int64_t total) {
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dq[QMAX];
  __shared__ double2 jq[JCMAX];
  const SysDev &S = sysv[sys];
  const int tid = threadIdx.x;
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  if (tid < S.Q) dq[tid] = control_value(S, alpha, carrier + S.carrier_off, tid, t);
  if (tid < S.njc) jq[tid] = jc_coef(S, tid, t);
  __syncthreads();
  const int64_t g = (int64_t)blockIdx.x * STREAM_BLOCK + tid;
  if (g >= total) return;
  const int64_t b = g / S.N2;
  const int64_t r = g - b * S.N2;
  const int i = (int)(r / S.N);
  const int jj = (int)(r - (int64_t)i * S.N);
  const uint64_t di = desc[S.tab_off + i], dj = desc[S.tab_off + jj];
  const double gam = diag_rate(S, di, dj);
  const double dE = Etab[S.tab_off + i] - Etab[S.tab_off + jj];
  const double2 *xs = x + b * S.N2;
  const double2 acc = offdiag_all<ADJ>(S, di, dj, r, dq, jq, sq, [&](int64_t idx) { return xs[idx]; });
  y[g] = cadd(acc, cmul(diag_coef(gam, dE, ADJ), xs[r]));
}

int launch_apply(const lb_plan *p, int sys, double t, const double *alpha, const double2 *x,
                 double2 *y, int B, bool adj, int tile_opt, int ki_opt, hipStream_t st) {
  const int64_t total = (int64_t)B * p->sys[sys].N2;
  if (total == 0) return LB_OK;
  if (tile_opt && (tile_ki(p, sys, ki_opt) > 0 || (tile_opt == 2 && split_kl(p, sys) > 0)))
    return launch_tile_apply(p, sys, B, adj, alpha, t, x, y, tile_opt, ki_opt, st);
  const int64_t nblk = (total + STREAM_BLOCK - 1) / STREAM_BLOCK;
  if (adj)
    hipLaunchKernelGGL(apply_kernel<true>, dim3((unsigned)nblk), dim3(STREAM_BLOCK), 0, st,
                       p->d_sys, sys, t, alpha, p->d_carrier, p->d_E, p->d_desc, x, y, total);
  else
    hipLaunchKernelGGL(apply_kernel<false>, dim3((unsigned)nblk), dim3(STREAM_BLOCK), 0, st,
                       p->d_sys, sys, t, alpha, p->d_carrier, p->d_E, p->d_desc, x, y, total);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

__device__ __forceinline__ int find_segment(const StreamSeg *segs, int nseg, int64_t blk) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ----------------------------------------------------------------------------
// Gradient integrands of one step for streamed systems (App. B eq.
// reducedgradient):  zh = (qh^j + qh^{j+1})/2 is the adjoint stage vector
// (written by the last sweep of the adjoint step), z = (q^j + q^{j+1})/2 the
// forward one.  Per-block partial sums.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(STREAM_BLOCK) void stream_grad_kernel(
    const SysDev *__restrict__ sysv, const StreamSeg *__restrict__ segs, int nseg,
    const uint64_t *__restrict__ desc, const double2 *__restrict__ zh,
    const double2 *__restrict__ q0, const double2 *__restrict__ q1, double *__restrict__ gpart) {
  __shared__ double sq[SQRT_TABLE];
  __shared__ int sseg;
  __shared__ double red[STREAM_BLOCK / 64][2 * QMAX];
  const int tid = threadIdx.x;
  if (tid == 0) sseg = find_segment(segs, nseg, blockIdx.x);
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  __syncthreads();
  const StreamSeg &sg = segs[sseg];
  const SysDev &S = sysv[sg.sys];
  const int64_t local = ((int64_t)blockIdx.x - sg.blk0) * STREAM_BLOCK + tid;
  const bool ok = local < sg.count;
  const int64_t b = ok ? local / S.N2 : 0;
  const int64_t r = ok ? local - b * S.N2 : 0;
  const int i = (int)(r / S.N);
  const int jj = (int)(r - (int64_t)i * S.N);
  const uint64_t di = desc[S.tab_off + i], dj = desc[S.tab_off + jj];
  const int64_t base = sg.off + b * S.N2;
  const double2 z = ok ? cscale(0.5, cadd(q0[base + r], q1[base + r])) : make_double2(0.0, 0.0);
  const int lane = tid & 63, wv = tid >> 6;
  for (int q = 0; q < S.Q; ++q) {
    double gp = 0.0, gq = 0.0;
    if (ok)
      grad_term(S, q, di, dj, r, z, sq, [&](int64_t idx) { return zh[base + idx]; }, gp, gq);
    gp = wave_sum<64>(gp);
    gq = wave_sum<64>(gq);
    if (lane == 0) {
      red[wv][2 * q] = gp;
      red[wv][2 * q + 1] = gq;
    }
  }
  __syncthreads();
  if (tid < 2 * S.Q) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < STREAM_BLOCK / 64; ++w) v += red[w][tid];
    gpart[(int64_t)blockIdx.x * 2 * QMAX + tid] = v;
  }
}

int launch_stream_grad(const lb_plan *p, const StreamSeg *d_segs, int nseg, int64_t nblk,
                       const double2 *zh, const double2 *q0, const double2 *q1, double *gpart,
                       hipStream_t st) {
  if (nblk == 0) return LB_OK;
  hipLaunchKernelGGL(stream_grad_kernel, dim3((unsigned)nblk), dim3(STREAM_BLOCK), 0, st, p->d_sys,
                     d_segs, nseg, p->d_desc, zh, q0, q1, gpart);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// Sum the block partials of each segment into gstep[s][j][2Q] in two fixed-
// order passes: FIN_SPLIT workgroups per segment each reduce a contiguous
// range of partial rows (one row of 2 QMAX doubles per thread and pass, so
// that a wavefront reads consecutive rows), then one workgroup per segment
// adds the FIN_SPLIT results.  Several steps are reduced in one launch
// (grid z / y: slot z holds step jtop - z), each in the same order as alone.
constexpr int FIN_SPLIT = 64;

__global__ __launch_bounds__(256) void stream_grad_partial_kernel(
    const SysDev *__restrict__ sysv, const StreamSeg *__restrict__ segs,
    const double *__restrict__ gpart, int64_t slot_stride, double *__restrict__ gfin,
    int64_t fin_stride, int64_t rows) {
  __shared__ double red[4][2 * QMAX];
  gpart += (int64_t)blockIdx.z * slot_stride;
  gfin += (int64_t)blockIdx.z * fin_stride;
  const StreamSeg &sg = segs[blockIdx.x];
  const int Q2 = 2 * sysv[sg.sys].Q;
  // rows > 0: one segment whose partial rows start at 0 (block-tiled kernel)
  const int64_t nb = rows > 0 ? rows : (sg.count + STREAM_BLOCK - 1) / STREAM_BLOCK;
  const int64_t row0 = rows > 0 ? 0 : sg.blk0;
  const int64_t per = (nb + FIN_SPLIT - 1) / FIN_SPLIT;
  const int64_t k0 = (int64_t)blockIdx.y * per;
  const int64_t k1 = k0 + per < nb ? k0 + per : nb;
  const int tid = threadIdx.x;
  double v[2 * QMAX];
#pragma unroll
  for (int c = 0; c < 2 * QMAX; ++c) v[c] = 0.0;
  for (int64_t k = k0 + tid; k < k1; k += 256) {
    const double *row = gpart + (row0 + k) * 2 * QMAX;
#pragma unroll
    for (int c = 0; c < 2 * QMAX; ++c)
      if (c < Q2) v[c] += row[c];
  }
#pragma unroll
  for (int c = 0; c < 2 * QMAX; ++c) {
    if (c >= Q2) break;
    const double w = wave_sum<64>(v[c]);
    if ((tid & 63) == 0) red[tid >> 6][c] = w;
  }
  __syncthreads();
  if (tid < Q2)
    gfin[((int64_t)blockIdx.x * FIN_SPLIT + blockIdx.y) * 2 * QMAX + tid] =
        red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

__global__ __launch_bounds__(64) void stream_grad_finalize_kernel(
    const SysDev *__restrict__ sysv, const StreamSeg *__restrict__ segs, int jtop,
    const double *__restrict__ gfin, int64_t fin_stride, double *__restrict__ gstep) {
  const int j = jtop - (int)blockIdx.y;
  gfin += (int64_t)blockIdx.y * fin_stride;
  const StreamSeg &sg = segs[blockIdx.x];
  const SysDev &S = sysv[sg.sys];
  const int c = threadIdx.x;
  if (c >= 2 * S.Q) return;
  double v = 0.0;
  for (int g = 0; g < FIN_SPLIT; ++g) v += gfin[((int64_t)blockIdx.x * FIN_SPLIT + g) * 2 * QMAX + c];
  gstep[2 * S.ctab_off + (int64_t)j * 2 * S.Q + c] = v;
}

size_t stream_grad_fin_doubles(int nseg) { return (size_t)std::max(nseg, 1) * FIN_SPLIT * 2 * QMAX; }

int launch_stream_grad_finalize(const lb_plan *p, const StreamSeg *d_segs, int nseg, int jtop,
                                int nsteps, const double *gpart, int64_t slot_stride, double *gfin,
                                double *gstep, int64_t rows, hipStream_t st) {
  if (nseg == 0 || nsteps == 0) return LB_OK;
  if (nsteps > 65535) return fail(LB_EINVAL, "too many steps in one gradient reduction");
  const int64_t fin_stride = (int64_t)stream_grad_fin_doubles(nseg);
  hipLaunchKernelGGL(stream_grad_partial_kernel, dim3(nseg, FIN_SPLIT, nsteps), dim3(256), 0, st,
                     p->d_sys, d_segs, gpart, slot_stride, gfin, fin_stride, rows);
  LBX_HIP(hipGetLastError());
  hipLaunchKernelGGL(stream_grad_finalize_kernel, dim3(nseg, nsteps), dim3(64), 0, st, p->d_sys, d_segs,
                     jtop, gfin, fin_stride, gstep);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// ----------------------------------------------------------------------------
// Adjoint terminal condition (App. B): qh = (beta_i/M) dJ/d(conj q), times
// the weight gscale[s] of the system's objective when gscale is given (the
// incoming gradient of a backward pass; the adjoint is linear in it).
//   J_Frob: rho(T) - rho_tar;   J_Tr: -rho_tar;   J_Nm: the observable N_m.
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(STREAM_BLOCK) void terminal_kernel(
    const SysDev *__restrict__ sysv, const StreamSeg *__restrict__ segs, int nseg, int kind,
    const double2 *__restrict__ rhoT, const double2 *__restrict__ rhotar,
    const double *__restrict__ beta, const int32_t *__restrict__ seg_state0,
    const double *__restrict__ gscale, double2 *__restrict__ qh) {
  __shared__ int sseg;
  if (threadIdx.x == 0) sseg = find_segment(segs, nseg, blockIdx.x);
  __syncthreads();
  const StreamSeg &sg = segs[sseg];
  const SysDev &S = sysv[sg.sys];
  const int64_t local = ((int64_t)blockIdx.x - sg.blk0) * STREAM_BLOCK + threadIdx.x;
  if (local >= sg.count) return;
  const int64_t b = local / S.N2;
  const double wgt = beta[seg_state0[sseg] + b] / (double)sg.nstates * (gscale ? gscale[sg.sys] : 1.0);
  const int64_t e = sg.off + local;
  const double2 t = rhotar[sg.boff + local];
  qh[e] = kind == LB_J_FROB ? cscale(wgt, csub(rhoT[e], t)) : cscale(kind == LB_J_NM ? wgt : -wgt, t);
}

int launch_terminal(const lb_plan *p, int kind, const StreamSeg *d_segs, int nseg, int64_t nblk,
                    const double2 *rhoT, const double2 *rhotar, const double *beta,
                    const int32_t *d_seg_state0, const double *gscale, double2 *qh, hipStream_t st) {
  if (nblk == 0) return LB_OK;
  hipLaunchKernelGGL(terminal_kernel, dim3((unsigned)nblk), dim3(STREAM_BLOCK), 0, st, p->d_sys,
                     d_segs, nseg, kind, rhoT, rhotar, beta, d_seg_state0, gscale, qh);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// ----------------------------------------------------------------------------
// Objective (Sec. III eqs. optimproblem, Jmeasure), two deterministic passes:
// per-state block partials of sum |rho - rho_tar|^2 (Frobenius) or
// Re sum conj(rho_tar) rho (trace), then per-system G.
// ----------------------------------------------------------------------------
constexpr int OBJ_PARTS = 64;

__global__ __launch_bounds__(256) void objective_partial_kernel(
    const SysDev *__restrict__ sysv, int kind, const double2 *__restrict__ rhoT,
    const double2 *__restrict__ rhotar, const int32_t *__restrict__ state_sys,
    const int64_t *__restrict__ state_off, double *__restrict__ partial) {
  __shared__ double red[4];
  const int state = blockIdx.y;
  const SysDev &S = sysv[state_sys[state]];
  const int64_t off = state_off[state];
  double v = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < S.N2; e += (int64_t)OBJ_PARTS * 256) {
    const double2 r = rhoT[off + e], t = rhotar[off + e];
    if (kind == LB_J_FROB) {
      const double dx = r.x - t.x, dy = r.y - t.y;
      v += dx * dx + dy * dy;
    } else {
      v += t.x * r.x + t.y * r.y;
    }
  }
  v = wave_sum<64>(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)state * OBJ_PARTS + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void objective_final_kernel(const SysDev *__restrict__ sysv, int nsys, int kind,
                                       const double *__restrict__ partial,
                                       const double *__restrict__ beta,
                                       const int32_t *__restrict__ sys_state0, double gamma2,
                                       const double *__restrict__ alpha, const double *__restrict__ pen,
                                       double *__restrict__ J, double *__restrict__ G,
                                       int32_t *__restrict__ status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  const SysDev &S = sysv[s];
  const int st0 = sys_state0[s], st1 = sys_state0[s + 1];
  double acc = 0.0;
  for (int st = st0; st < st1; ++st) {
    double v = 0.0;
    for (int k = 0; k < OBJ_PARTS; ++k) v += partial[(int64_t)st * OBJ_PARTS + k];
    const double Jst = kind == LB_J_FROB ? 0.5 * v : kind == LB_J_TR ? 1.0 - v : v;
    if (J) J[st] = Jst;
    acc += beta[st] * Jst;
  }
  double reg = 0.0;
  for (int k = 0; k < S.nalpha; ++k) {
    const double a = alpha[S.alpha_off + k];
    reg += a * a;
  }
  const int M = st1 - st0;
  const double g = (M > 0 ? acc / (double)M : 0.0) + 0.5 * gamma2 * reg + (pen ? pen[s] : 0.0);
  if (G) G[s] = g;
  if (status && M > 0 && !isfinite(g)) atomicOr(status, LB_STATUS_NONFINITE);
}

int launch_objective(const lb_plan *p, int kind, const double2 *rhoT, const double2 *rhotar,
                     const double *beta, const int32_t *d_state_sys, const int64_t *d_state_off,
                     const int32_t *d_sys_state0, int nstates, double gamma2, const double *alpha,
                     const double *pen, double *partial, double *J, double *G, int32_t *status,
                     hipStream_t st) {
  if (nstates > 0) {
    hipLaunchKernelGGL(objective_partial_kernel, dim3(OBJ_PARTS, nstates), dim3(256), 0, st,
                       p->d_sys, kind, rhoT, rhotar, d_state_sys, d_state_off, partial);
    LBX_HIP(hipGetLastError());
  }
  const int nsys = (int)p->sys.size();
  hipLaunchKernelGGL(objective_final_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, p->d_sys, nsys,
                     kind, partial, beta, d_sys_state0, gamma2, alpha, pen, J, G, status);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// ----------------------------------------------------------------------------
// Running penalty (Sec. III eq. optimproblem, gamma1 term) by the left
// rectangle rule: gamma1 (1/M) sum_i dt sum_{j<NT} beta(t_j) J(q_i^j), and
// its adjoint source gamma1 dt beta(t_j) (1/M) dJ/d(conj q^j) (App. B).  The
// sums are deterministic: every stream block owns one accumulator across the
// steps, every LDS-resident state a fixed set of chunk partials.
// ----------------------------------------------------------------------------
__global__ void penalty_table_kernel(const SysDev *__restrict__ sysv, int nsys, int NT, double gamma1, double a,
                                     double *__restrict__ ptab) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)nsys * NT) return;
  const SysDev &S = sysv[k / NT];
  const int j = (int)(k % NT);
  const double u = ((double)j * S.dt - S.T) / a;
  ptab[k] = gamma1 * S.dt * (exp(-(u * u)) / a);
}

int launch_penalty_table(const lb_plan *p, double gamma1, double a, double *ptab, hipStream_t st) {
  const int64_t n = (int64_t)p->sys.size() * p->NT;
  hipLaunchKernelGGL(penalty_table_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p->d_sys,
                     (int)p->sys.size(), p->NT, gamma1, a, ptab);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// Merit value of one entry: |q - t|^2 / 2 (J_Frob) or Re conj(t) q.
__device__ __forceinline__ double penalty_value(int kind, double2 q, double2 t) {
  if (kind == LB_J_FROB) {
    const double dx = q.x - t.x, dy = q.y - t.y;
    return 0.5 * (dx * dx + dy * dy);
  }
  return t.x * q.x + t.y * q.y;
}

// Sum over a 256-thread block, in a fixed order; valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double *red) {
  v = wave_sum<64>(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(STREAM_BLOCK) void penalty_accum_kernel(
    const SysDev *__restrict__ sysv, const StreamSeg *__restrict__ segs, int nseg, int kind, int NT, int j,
    const double2 *__restrict__ q, const double2 *__restrict__ rhotar, const double *__restrict__ ptab,
    double *__restrict__ acc) {
  static_assert(STREAM_BLOCK == 256, "block_sum256 assumes 256 threads");
  __shared__ int sseg;
  __shared__ double red[4];
  if (threadIdx.x == 0) sseg = find_segment(segs, nseg, blockIdx.x);
  __syncthreads();
  const StreamSeg &sg = segs[sseg];
  const int64_t local = ((int64_t)blockIdx.x - sg.blk0) * STREAM_BLOCK + threadIdx.x;
  const double v = local < sg.count ? penalty_value(kind, q[sg.off + local], rhotar[sg.boff + local]) : 0.0;
  const double b = block_sum256(v, red);
  if (threadIdx.x == 0) acc[blockIdx.x] += ptab[(int64_t)sg.sys * NT + j] * b;
}

int launch_penalty_accum(const lb_plan *p, int kind, const StreamSeg *d_segs, int nseg, int64_t nblk, int j,
                         const double2 *q, const double2 *rhotar, const double *ptab, double *acc,
                         hipStream_t st) {
  if (nblk == 0) return LB_OK;
  hipLaunchKernelGGL(penalty_accum_kernel, dim3((unsigned)nblk), dim3(STREAM_BLOCK), 0, st, p->d_sys, d_segs,
                     nseg, kind, p->NT, j, q, rhotar, ptab, acc);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

__global__ __launch_bounds__(256) void penalty_lds_kernel(const SysDev *__restrict__ sysv,
                                                          const LdsItem *__restrict__ items, int kind, int NT,
                                                          const double2 *__restrict__ hist,
                                                          const double2 *__restrict__ rhotar,
                                                          const double *__restrict__ ptab,
                                                          double *__restrict__ part) {
  __shared__ double red[4];
  const LdsItem it = items[blockIdx.x];
  const SysDev &S = sysv[it.sys];
  const int per = (NT + PEN_PARTS - 1) / PEN_PARTS;
  const int j0 = (int)blockIdx.y * per, j1 = min(NT, j0 + per);
  double v = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double2 *qj = hist + it.st_off + (int64_t)j * S.N2;
    double s = 0.0;
    for (int64_t e = threadIdx.x; e < S.N2; e += 256) s += penalty_value(kind, qj[e], rhotar[it.off + e]);
    v += ptab[(int64_t)it.sys * NT + j] * s;
  }
  const double b = block_sum256(v, red);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * PEN_PARTS + blockIdx.y] = b;
}

int launch_penalty_lds(const lb_plan *p, int kind, const LdsItem *d_items, int nitems, const double2 *hist,
                       const double2 *rhotar, const double *ptab, double *part, hipStream_t st) {
  if (nitems == 0) return LB_OK;
  hipLaunchKernelGGL(penalty_lds_kernel, dim3((unsigned)nitems, PEN_PARTS), dim3(256), 0, st, p->d_sys, d_items,
                     kind, p->NT, hist, rhotar, ptab, part);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

__global__ __launch_bounds__(256) void penalty_final_kernel(int kind, int NT, const int64_t *__restrict__ rng,
                                                            const double *__restrict__ acc,
                                                            const double *__restrict__ part,
                                                            const double *__restrict__ ptab,
                                                            const int32_t *__restrict__ sys_state0,
                                                            double *__restrict__ pen) {
  __shared__ double red[4];
  const int s = blockIdx.x;
  const int64_t b0 = rng[4 * s], nb = rng[4 * s + 1], i0 = rng[4 * s + 2], ni = rng[4 * s + 3];
  double v = 0.0;
  for (int64_t k = threadIdx.x; k < nb; k += 256) v += acc[b0 + k];
  for (int64_t k = threadIdx.x; k < ni * PEN_PARTS; k += 256) v += part[i0 * PEN_PARTS + k];
  const double tot = block_sum256(v, red);
  double w = 0.0;
  if (kind == LB_J_TR)
    for (int j = threadIdx.x; j < NT; j += 256) w += ptab[(int64_t)s * NT + j];
  const double wsum = block_sum256(w, red);
  if (threadIdx.x == 0) {
    const int M = sys_state0[s + 1] - sys_state0[s];
    // J_Tr = 1 - sum v: the constant integrates to sum_j ptab (times M / M).
    pen[s] = M == 0 ? 0.0 : (kind == LB_J_TR ? wsum - tot / (double)M : tot / (double)M);
  }
}

int launch_penalty_final(const lb_plan *p, int kind, const int64_t *d_rng, const double *acc,
                         const double *part, const double *ptab, const int32_t *d_sys_state0, double *pen,
                         hipStream_t st) {
  hipLaunchKernelGGL(penalty_final_kernel, dim3((unsigned)p->sys.size()), dim3(256), 0, st, kind, p->NT, d_rng,
                     acc, part, ptab, d_sys_state0, pen);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

__global__ __launch_bounds__(STREAM_BLOCK) void penalty_source_kernel(
    const StreamSeg *__restrict__ segs, int nseg, int kind, int NT, int j, const double2 *__restrict__ q,
    const double2 *__restrict__ rhotar, const double *__restrict__ ptab, const double *__restrict__ gscale,
    double2 *__restrict__ qh) {
  __shared__ int sseg;
  if (threadIdx.x == 0) sseg = find_segment(segs, nseg, blockIdx.x);
  __syncthreads();
  const StreamSeg &sg = segs[sseg];
  const int64_t local = ((int64_t)blockIdx.x - sg.blk0) * STREAM_BLOCK + threadIdx.x;
  if (local >= sg.count) return;
  const double w = ptab[(int64_t)sg.sys * NT + j] / (double)sg.nstates * (gscale ? gscale[sg.sys] : 1.0);
  const int64_t e = sg.off + local;
  const double2 t = rhotar[sg.boff + local];
  const double2 d = kind == LB_J_FROB ? csub(q[e], t) : (kind == LB_J_NM ? t : cscale(-1.0, t));
  qh[e] = cadd(qh[e], cscale(w, d));
}

int launch_penalty_source(const lb_plan *p, int kind, const StreamSeg *d_segs, int nseg, int64_t nblk, int j,
                          const double2 *q, const double2 *rhotar, const double *ptab, const double *gscale,
                          double2 *qh, hipStream_t st) {
  if (nblk == 0) return LB_OK;
  hipLaunchKernelGGL(penalty_source_kernel, dim3((unsigned)nblk), dim3(STREAM_BLOCK), 0, st, d_segs, nseg, kind,
                     p->NT, j, q, rhotar, ptab, gscale, qh);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// ----------------------------------------------------------------------------
// Gradient contraction (App. B eq. reducedgradient through the control
// parameterisation of eq. rotctrl):
//   dG/dRe alpha_q^{s,f} = dt sum_j 2pi S_s(t) [gp cos(W t) + gq sin(W t)] + gamma2 Re alpha
//   dG/dIm alpha_q^{s,f} = dt sum_j 2pi S_s(t) [-gp sin(W t) + gq cos(W t)] + gamma2 Im alpha
// with t = t_{j+1/2}, W = 2 pi Omega_q^f, gp/gq the per-step integrands.  With
// gscale (a backward pass) the integrands already carry the system's weight
// through the terminal condition, and the Tikhonov term is scaled by it.
// ----------------------------------------------------------------------------
// One workgroup per (system, q, s, f): its threads take the steps of the
// spline's support in turn (one sincos per step for both the Re and the Im
// coefficient), and the workgroup sums them in a fixed order.
constexpr int CONTRACT_BLOCK = 256;

__global__ __launch_bounds__(CONTRACT_BLOCK) void grad_contract_kernel(
    const SysDev *__restrict__ sysv, int nsys, const double *__restrict__ gstep,
    const double *__restrict__ alpha, const double *__restrict__ carrier, double gamma2,
    const double *__restrict__ gscale, double *__restrict__ grad) {
  __shared__ double red[CONTRACT_BLOCK / 64][2];
  const int64_t k = 2 * (int64_t)blockIdx.x;  // the Re coefficient; k + 1 is the Im one
  int s = 0;
  while (s + 1 < nsys && sysv[s + 1].alpha_off <= k) ++s;
  const SysDev &S = sysv[s];
  const int64_t loc = k - S.alpha_off;
  const int f = (int)((loc / 2) % S.Nf);
  const int sp = (int)((loc / (2 * S.Nf)) % S.Ns);
  const int q = (int)(loc / (2 * S.Nf * S.Ns));
  const double Om = TWO_PI * carrier[S.carrier_off + q * S.Nf + f];
  int j0 = (int)floor((sp - 2.0) * S.dtau / S.dt - 0.5) - 1;
  int j1 = (int)ceil((sp + 1.0) * S.dtau / S.dt) + 1;
  j0 = j0 < 0 ? 0 : j0;
  j1 = j1 > S.NT - 1 ? S.NT - 1 : j1;
  double are = 0.0, aim = 0.0;
  for (int j = j0 + (int)threadIdx.x; j <= j1; j += CONTRACT_BLOCK) {
    const double t = ((double)j + 0.5) * S.dt;
    const double B = bspline2(t / S.dtau - (double)sp + 0.5);
    if (B == 0.0) continue;
    double sn, cs;
    sincos(Om * t, &sn, &cs);
    const double gp = gstep[2 * S.ctab_off + (int64_t)j * 2 * S.Q + 2 * q];
    const double gq = gstep[2 * S.ctab_off + (int64_t)j * 2 * S.Q + 2 * q + 1];
    are += B * (gp * cs + gq * sn);
    aim += B * (-gp * sn + gq * cs);
  }
  are = wave_sum<64>(are);
  aim = wave_sum<64>(aim);
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6][0] = are;
    red[threadIdx.x >> 6][1] = aim;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < CONTRACT_BLOCK / 64; ++w) v += red[w][threadIdx.x];
    const double gw = gscale ? gscale[s] : 1.0;
    grad[k + threadIdx.x] = TWO_PI * S.dt * v + gw * gamma2 * alpha[k + threadIdx.x];
  }
}

int launch_grad_contract(const lb_plan *p, const double *gstep, const double *alpha,
                         double gamma2, const double *gscale, double *grad, hipStream_t st) {
  const int nsys = (int)p->sys.size();
  const int64_t total = p->sys[nsys - 1].alpha_off + p->sys[nsys - 1].nalpha;
  if (total == 0) return LB_OK;
  hipLaunchKernelGGL(grad_contract_kernel, dim3((unsigned)(total / 2)), dim3(CONTRACT_BLOCK), 0, st,
                     p->d_sys, nsys, gstep, alpha, p->d_carrier, gamma2, gscale, grad);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

}  // namespace lbx
