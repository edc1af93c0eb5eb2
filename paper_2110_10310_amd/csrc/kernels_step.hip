// Stage-solve sweeps of the implicit-midpoint steps of streamed systems
// (states in HBM), App. A eqs. IMR and linsystem_primal; App. B eq.
// linsystem_adjoint for the adjoint.  One launch per sweep, one unit per
// workgroup; the number of sweeps of every step is decided on the device.
//
// Stage solve.  (I - h M) z = q with h = dt/2 and M = D + O is solved in
// delta form, z = q + delta:  delta <- w (h D q + h O (q + delta)),
// w = (1 - h D)^-1.  Since Re D <= 0, |w| <= 1 and the map contracts in the
// max norm with a factor theta_j <= h sum_q (2 |d_q| c_q + (n_q - 1)/T1_q)
// (control_table_kernel).  After a first sweep delta0 -> delta1 the error obeys
//   |delta1 - delta*| <= theta/(1 - theta) |delta1 - delta0|,
// and every further sweep multiplies the bound by theta; a step takes at
// least two sweeps and otherwise the fewest that bring the bound below
// tol * max|q|.  Sweep 0 folds its workgroup maxima of |delta1 - delta0| and
// |q| into LB_STEP_SLOTS slots per system with atomic maxima (exact, so the
// order does not matter); a one-wavefront count kernel reduces those slots
// into the step's count K, and every workgroup of a later sweep reads K,
// runs if its sweep index is below K, takes the update if it is K - 1, and
// returns at once otherwise.  The host launches a fixed number of sweeps per
// step; a step that would need more raises LB_STATUS_RETRY, and the library
// repeats the call with counts known on the host (A.apriori: every launched
// sweep runs).
//
// Start.  A step starts from delta0 = 0 (z = q) or from an extrapolation of
// the converged increments of the previous steps of the same pass.  For
// M = D alone the increments obey delta_{j+1} = R delta_j with the diagonal
// Cayley factor R = (1 + h D) w, so the extrapolation is polynomial in the
// frame that factor rotates away: with the history delta_n, ..., delta_{n-m+1}
//   delta0_{n+1} = sum_{k<m} (-1)^k C(m, k+1) R^{k+1} delta_{n-k}
// (order m - 1 in t; the controls are piecewise quadratic in t).  The last
// sweep of a step forms that start for the next step, writes it as the next
// step's first iterate, and files its own increment in a ring of H buffers.
//
// Update.  q^{j+1} = q^j + dt M z = q^j + 2 delta (h M z = z - q = delta).
// The adjoint step has the same form with M^+ and also writes its stage
// vector zh = q + delta for the gradient integrands.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbx_host.hpp"
#include "tile_unit.hpp"

namespace lbx {

namespace {

// Total sweeps of a stage solve after a first sweep that changed the iterate
// by e1 (max norm), with |q| <= qmax: at least two, at most kcap + 1.
__device__ __forceinline__ int stage_sweeps(double theta, double ratio, double e1, double qmax, double tol,
                                            int kcap) {
  double r = ratio * e1;
  const double lim = tol * qmax;
  int k = 0;
  while (r > lim && k < kcap) {
    r *= theta;
    ++k;
  }
  return 1 + (k > 1 ? k : 1);
}

// Order-preserving bits of a non-negative double (NaN orders above every
// finite value, so a NaN iterate still yields a count).
__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ __forceinline__ double bdbl(unsigned long long b) { return __longlong_as_double((long long)b); }

// Maximum over the workgroup of two non-negative values, valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ void block_max2(double &a, double &b, double (*red)[BLOCK / 64]) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off, 64));
    b = fmax(b, __shfl_xor(b, off, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = a;
    red[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 1; k < BLOCK / 64; ++k) {
      a = fmax(a, red[0][k]);
      b = fmax(b, red[1][k]);
    }
  }
}

// Slots of system `sys` for the step with parity `par`: LB_STEP_SLOTS maxima
// of |delta1 - delta0|, then LB_STEP_SLOTS maxima of |q|.
__device__ __forceinline__ unsigned long long *slot_base(const StepArgs &A, int par, int sys) {
  return A.slots + ((int64_t)par * A.nsys + sys) * 2 * LB_STEP_SLOTS;
}

// Sweeps of the current step of system `sys` (written by step_count_kernel).
__device__ __forceinline__ int step_sweeps_of(const StepArgs &A, int sys) {
  return A.kstep[(int64_t)A.par * A.nsys + sys];
}

__device__ __forceinline__ double2 cfma(double2 acc, double c, double2 r, double2 d) {
  const double2 rd = cmul(r, d);
  return make_double2(acc.x + c * rd.x, acc.y + c * rd.y);
}

// Start of the next step from the history (see the file comment): dn is this
// step's increment delta_n, R the diagonal Cayley factor, ring slot
// (n - k) mod H holds delta_{n-k} for k = 1 .. m-1.
constexpr int HMAX = 4;

__device__ __forceinline__ double2 next_start(double2 dn, double2 R, int m, int n, int H,
                                              const double2 *__restrict__ ring, int64_t stride, int64_t e) {
  double2 Rk = R;
  double binom = (double)m;  // C(m, 1)
  double2 pred = cfma(make_double2(0.0, 0.0), binom, Rk, dn);
#pragma unroll
  for (int k = 1; k < HMAX; ++k) {
    if (k >= m) break;
    binom = binom * (double)(m - k) / (double)(k + 1);  // C(m, k+1)
    Rk = cmul(Rk, R);
    const int slot = ((n - k) % H + H) % H;
    pred = cfma(pred, (k & 1) ? -binom : binom, Rk, ring[(int64_t)slot * stride + e]);
  }
  return pred;
}

// The output of one entry of sweep kk (first: kk == 0; last: takes the update).
struct SweepOut {
  double2 *zo;
  bool first, last;
  double e1 = 0.0, qm = 0.0;
};

template <bool ADJ>
__device__ __forceinline__ void sweep_entry(const StepArgs &A, SweepOut &so, int64_t e, double h, double gam,
                                            double dE, double2 acc, double2 own) {
  const double2 qv = A.q[e];
  const double2 D = diag_coef(gam, dE, ADJ);
  const double2 w = stage_weight(h, gam, dE, ADJ);
  const double2 hdq = cscale(h, cmul(D, qv));
  const double2 dn = cmul(w, make_double2(hdq.x + h * acc.x, hdq.y + h * acc.y));
  if (so.first) {
    const double2 d0 = csub(own, qv);
    so.e1 = fmax(so.e1, fabs(dn.x - d0.x) + fabs(dn.y - d0.y));
    so.qm = fmax(so.qm, fmax(fabs(qv.x), fabs(qv.y)));
  }
  if (!so.last) {
    so.zo[e] = cadd(qv, dn);
    return;
  }
  const double2 qn = make_double2(qv.x + 2.0 * dn.x, qv.y + 2.0 * dn.y);
  A.out[e] = qn;
  if (ADJ && A.zh) A.zh[e] = cadd(qv, dn);
  if (A.znext) {
    const double2 R = cmul(make_double2(1.0 + h * D.x, h * D.y), w);
    A.znext[e] = cadd(qn, next_start(dn, R, A.m, A.n, A.H, A.ring, A.ring_stride, e));
    A.ring[(int64_t)(A.n % A.H) * A.ring_stride + e] = dn;
  }
}

// The iterate sweep kk reads: the start for kk = 0, then the output of kk - 1.
__device__ __forceinline__ const double2 *sweep_input(const StepArgs &A, int kk) {
  if (kk == 0) return A.zstart ? A.zstart : A.q;
  return (kk & 1) ? A.z0 : A.z1;
}

}  // namespace

// ----------------------------------------------------------------------------
// Block-tiled sweep of one system of equal-level subsystems.
// ----------------------------------------------------------------------------
template <int NL, int QC, int KR, int KC, bool ADJ, int BLOCK>
__global__ __launch_bounds__(BLOCK) void sweep_tile_kernel(StepArgs A, int kk) {
  extern __shared__ double2 tileb[];
  __shared__ double red[2][BLOCK / 64];
  const int64_t per = (A.units + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= A.units) return;
  const SysDev &S = A.sysv[A.sys];
  int K = 2;
  if (kk > 0) {
    K = step_sweeps_of(A, A.sys);
    if (kk >= K) return;  // this step's solve is done (uniform per launch)
  }
  const int lane = threadIdx.x & 63;
  double2 dv = make_double2(0.0, 0.0);
  if (lane < QC) dv = A.ctab[S.ctab_off + (int64_t)A.j * QC + lane - A.cshift];
  double da[QC], db[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    da[q] = tile::lane_d(dv.x, q);
    db[q] = tile::lane_d(dv.y, q);
  }
  SweepOut so;
  so.first = kk == 0;
  so.last = kk > 0 && kk == K - 1;
  so.zo = (kk & 1) ? A.z1 : A.z0;
  const double h = S.h;
  tile::tile_unit<NL, QC, KR, KC, ADJ, BLOCK>(S, lb, sweep_input(A, kk), tileb, da, db, A.Etab + S.tab_off, false,
                                              [&](const tile::Entry &en) {
                                                sweep_entry<ADJ>(A, so, en.e, h, en.gam, en.dE, en.acc, en.own);
                                              });
  if (so.first) {
    block_max2<BLOCK>(so.e1, so.qm, red);
    if (threadIdx.x == 0) {
      unsigned long long *sl = slot_base(A, A.par, A.sys);
      atomicMax(&sl[blockIdx.x % LB_STEP_SLOTS], dbits(so.e1));
      atomicMax(&sl[LB_STEP_SLOTS + blockIdx.x % LB_STEP_SLOTS], dbits(so.qm));
    }
  }
}

// ----------------------------------------------------------------------------
// Generic sweep over the segments of a streamed batch (any systems): one
// entry per thread, neighbours read directly from the batch.  Every segment
// runs its own sweep count.
// ----------------------------------------------------------------------------
__device__ __forceinline__ int find_seg(const StreamSeg *segs, int nseg, int64_t blk) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <bool ADJ>
__global__ __launch_bounds__(STREAM_BLOCK) void sweep_generic_kernel(StepArgs A, int kk) {
  constexpr int BLOCK = STREAM_BLOCK;
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dq[QMAX];
  __shared__ double red[2][BLOCK / 64];
  const int tid = threadIdx.x;
  const int64_t u = blockIdx.x;
  const int sgi = find_seg(A.segs, A.nseg, u);
  const StreamSeg &sg = A.segs[sgi];
  const SysDev &S = A.sysv[sg.sys];
  int K = 2;
  if (kk > 0) {
    K = step_sweeps_of(A, sg.sys);
    if (kk >= K) return;  // uniform per workgroup
  }
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  if (tid < S.Q) dq[tid] = A.ctab[S.ctab_off + (int64_t)A.j * S.Q + tid - A.cshift];
  __syncthreads();
  SweepOut so;
  so.first = kk == 0;
  so.last = kk > 0 && kk == K - 1;
  so.zo = (kk & 1) ? A.z1 : A.z0;
  const double2 *zin = sweep_input(A, kk);
  const int64_t local = (u - sg.blk0) * BLOCK + tid;
  if (local < sg.count) {
    const int64_t b = local / S.N2;
    const int64_t r = local - b * S.N2;
    const int i = (int)(r / S.N);
    const int jj = (int)(r - (int64_t)i * S.N);
    const uint64_t di = A.desc[S.tab_off + i], dj = A.desc[S.tab_off + jj];
    const int64_t base = sg.off + b * S.N2;
    const double2 acc = offdiag<ADJ>(S, di, dj, r, dq, sq, [&](int64_t idx) { return zin[base + idx]; });
    sweep_entry<ADJ>(A, so, base + r, S.h, diag_rate(S, di, dj), A.Etab[S.tab_off + i] - A.Etab[S.tab_off + jj],
                     acc, zin[base + r]);
  }
  if (so.first) {
    block_max2<BLOCK>(so.e1, so.qm, red);
    if (tid == 0) {
      unsigned long long *sl = slot_base(A, A.par, sg.sys);
      const int k = (int)((u - sg.blk0) % LB_STEP_SLOTS);
      atomicMax(&sl[k], dbits(so.e1));
      atomicMax(&sl[LB_STEP_SLOTS + k], dbits(so.qm));
    }
  }
}

// Sweep count of the current step of every streamed system, after sweep 0:
// workgroup g takes segment g, reduces the system's slots (one per lane),
// writes the count, raises status bits, adds the count to kout and clears
// the slots that the next step's sweep 0 fills.
__global__ __launch_bounds__(64) void step_count_kernel(StepArgs A) {
  const int sys = A.segs[blockIdx.x].sys;
  const int lane = threadIdx.x;
  unsigned long long *sl = slot_base(A, A.par, sys);
  double e1 = bdbl(sl[lane]), qm = bdbl(sl[LB_STEP_SLOTS + lane]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    e1 = fmax(e1, __shfl_xor(e1, off, 64));
    qm = fmax(qm, __shfl_xor(qm, off, 64));
  }
  unsigned long long *nx = slot_base(A, A.par ^ 1, sys);
  nx[lane] = 0ull;
  nx[LB_STEP_SLOTS + lane] = 0ull;
  if (lane != 0) return;
  const double2 tt = A.ttab[(int64_t)sys * A.NT + A.j - A.tshift];
  int K = A.L;
  int bits = 0;
  if (!A.apriori) {
    K = stage_sweeps(tt.x, tt.y, e1, qm, A.tol, A.kcap);
    if (K > A.L) {
      bits |= LB_STATUS_RETRY;
      K = A.L;
    }
  }
  if (!(tt.x < 0.5)) bits |= LB_STATUS_THETA;
  if (bits && A.status) atomicOr(A.status, bits);
  A.kstep[(int64_t)A.par * A.nsys + sys] = K;
  if (A.kout) A.kout[(int64_t)sys * A.NT + A.j] += K;
}

// Clears the slots of both parities of every system (start of a call).
__global__ void slots_clear_kernel(unsigned long long *slots, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    slots[i] = 0ull;
}

int launch_slots_clear(unsigned long long *slots, int nsys, hipStream_t st) {
  const int64_t n = (int64_t)2 * nsys * 2 * LB_STEP_SLOTS;
  hipLaunchKernelGGL(slots_clear_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, st,
                     slots, n);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
namespace {

template <int NL, int QC, int KR, int KC, int BLOCK>
int sweep_tile_launch(const lb_plan *p, StepArgs &A, int kk, bool adj, hipStream_t st) {
  using Sh = tile::Shape<NL, QC, KR, KC, BLOCK>;
  A.units = tile::tile_units(p->sys[A.sys].N, Sh::TR, Sh::TC, A.B);
  const size_t shmem = Sh::lds_bytes();
  const void *f = adj ? (const void *)sweep_tile_kernel<NL, QC, KR, KC, true, BLOCK>
                      : (const void *)sweep_tile_kernel<NL, QC, KR, KC, false, BLOCK>;
  LBX_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const dim3 grid((unsigned)(((A.units + 7) / 8) * 8));
  if (adj)
    hipLaunchKernelGGL((sweep_tile_kernel<NL, QC, KR, KC, true, BLOCK>), grid, dim3(BLOCK), shmem, st, A, kk);
  else
    hipLaunchKernelGGL((sweep_tile_kernel<NL, QC, KR, KC, false, BLOCK>), grid, dim3(BLOCK), shmem, st, A, kk);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

}  // namespace

namespace {

int sweep_only(const lb_plan *p, StepArgs &A, int kk, bool adj, int tile_sys, int tile_k, hipStream_t st) {
  if (tile_sys >= 0) {
    const SysDev &S = p->sys[tile_sys];
    const int nl = S.nlev[0];
    A.sys = tile_sys;
#define X(NL_, Q_, R_, C_, T_) \
  if (nl == NL_ && S.Q == Q_ && tile_k == 10 * R_ + C_) return sweep_tile_launch<NL_, Q_, R_, C_, T_>(p, A, kk, adj, st);
    LBX_TILE_SHAPES(X)
#undef X
    return fail(LB_EUNSUPPORTED, "no block-tiled sweep kernel for this system");
  }
  if (A.nblk == 0) return LB_OK;
  if (adj)
    hipLaunchKernelGGL(sweep_generic_kernel<true>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, kk);
  else
    hipLaunchKernelGGL(sweep_generic_kernel<false>, dim3((unsigned)A.nblk), dim3(STREAM_BLOCK), 0, st, A, kk);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

}  // namespace

int launch_sweep(const lb_plan *p, StepArgs &A, int kk, bool adj, int tile_sys, int tile_k, hipStream_t st) {
  if (A.H > HMAX) return fail(LB_EINVAL, "increment history longer than the kernels keep");
  if (int rc = sweep_only(p, A, kk, adj, tile_sys, tile_k, st)) return rc;
  if (kk == 0 && A.nseg > 0) {
    hipLaunchKernelGGL(step_count_kernel, dim3((unsigned)A.nseg), dim3(64), 0, st, A);
    LBX_HIP(hipGetLastError());
  }
  return LB_OK;
}

}  // namespace lbx
