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
// and every further sweep multiplies the bound by theta; a step takes the
// fewest sweeps that bring the bound below tol * max|q|.  A step whose first
// sweep suffices (its start was within the bound) is finished by
// stage_finish_kernel, which writes the step's outputs from that sweep's
// iterate without another pass over the neighbours.  Sweep 0 folds its
// workgroup maxima of |delta1 - delta0| and
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
// by e1 (max norm), with |q| <= qmax: at least one, at most kcap + 1.
__device__ __forceinline__ int stage_sweeps(double theta, double ratio, double e1, double qmax, double tol,
                                            int kcap) {
  double r = ratio * e1;
  const double lim = tol * qmax;
  int k = 0;
  while (r > lim && k < kcap) {
    r *= theta;
    ++k;
  }
  return 1 + k;
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
constexpr int HMAX = 6;

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

// What the last sweep of a step writes for entry e, from its increment dn:
// q^{j+1} = q + 2 dn, the stage vector q + dn (adjoint), and the next step's
// start and the increment history.
template <bool ADJ>
__device__ __forceinline__ void step_output(const StepArgs &A, int64_t e, double h, double2 D, double2 w, double2 qv,
                                            double2 dn) {
  const double2 qn = make_double2(qv.x + 2.0 * dn.x, qv.y + 2.0 * dn.y);
  A.out[e] = qn;
  if (ADJ && A.zh) A.zh[e] = cadd(qv, dn);
  if (A.znext) {
    const double2 R = cmul(make_double2(1.0 + h * D.x, h * D.y), w);
    A.znext[e] = cadd(qn, next_start(dn, R, A.m, A.n, A.H, A.ring, A.ring_stride, e));
    A.ring[(int64_t)(A.n % A.H) * A.ring_stride + e] = dn;
  }
}

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
  step_output<ADJ>(A, e, h, D, w, qv, dn);
}

// The iterate sweep kk reads: the start for kk = 0, then the output of kk - 1.
__host__ __device__ __forceinline__ const double2 *sweep_input(const StepArgs &A, int kk) {
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
    if (ADJ && A.gpart && kk == K - 1) return;  // sweep_tile_grad_kernel takes it
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

// Last sweep of a block-tiled adjoint step together with the step's gradient
// integrands (App. B eq. reducedgradient), which read the stage vector at the
// neighbours the sweep loads anyway.  The stage vector of the integrands is
// the sweep's input iterate (after K - 1 sweeps) instead of the converged one:
// the two differ by at most the solve's bound one sweep earlier, about
// tol / theta relative.  Runs only when kk is the step's last sweep (the plain
// kernel skips that one), writes the step's update like any last sweep, and
// one row of 2 Q partial sums per unit into A.gpart in a fixed order.
template <int NL, int QC, int KR, int KC, int BLOCK>
__global__ __launch_bounds__(BLOCK) void sweep_tile_grad_kernel(StepArgs A, int kk) {
  extern __shared__ double2 tileb[];
  __shared__ double red[BLOCK / 64][2 * QC];
  const int64_t per = (A.units + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= A.units) return;
  const SysDev &S = A.sysv[A.sys];
  const int K = step_sweeps_of(A, A.sys);
  if (kk != K - 1) return;  // uniform per launch
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
  so.first = false;
  so.last = true;
  so.zo = (kk & 1) ? A.z1 : A.z0;
  tile::GradAcc<QC> ga;
  ga.q0 = A.gq0;
  ga.q1 = A.gq1;
#pragma unroll
  for (int q = 0; q < QC; ++q) ga.p[q] = ga.q[q] = 0.0;
  const double h = S.h;
  tile::tile_unit<NL, QC, KR, KC, true, BLOCK, true>(
      S, lb, sweep_input(A, kk), tileb, da, db, A.Etab + S.tab_off, false,
      [&](const tile::Entry &en) { sweep_entry<true>(A, so, en.e, h, en.gam, en.dE, en.acc, en.own); }, &ga);
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const double a = wave_sum<64>(ga.p[q]), c = wave_sum<64>(ga.q[q]);
    if (lane == 0) {
      red[wv][2 * q] = a;
      red[wv][2 * q + 1] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * QC) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) v += red[w][threadIdx.x];
    A.gpart[lb * 2 * QMAX + threadIdx.x] = v;
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
  __shared__ double2 jq[JCMAX];
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
  if (tid < S.njc) jq[tid] = jc_coef(S, tid, ((double)A.j + 0.5) * S.dt);
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
    const double2 acc =
        offdiag_all<ADJ>(S, di, dj, r, dq, jq, sq, [&](int64_t idx) { return zin[base + idx]; });
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

// The outputs of a step whose stage solve converged in its first sweep
// (count 1), for every streamed system with that count: sweep 0 left
// z = q + delta in z0, and this writes what a last sweep writes
// (step_output) without another pass over the neighbours.  delta is
// recovered as z - q, exact where |delta| << |q| and otherwise within one
// rounding of z.
// A bounded grid walks the STREAM_BLOCK-entry units, so that the launch costs
// little when no system has count 1.
template <bool ADJ>
__global__ __launch_bounds__(STREAM_BLOCK) void stage_finish_kernel(StepArgs A) {
  if (A.nseg == 1 && step_sweeps_of(A, A.segs[0].sys) != 1) return;  // one system: one test
  for (int64_t u = blockIdx.x; u < A.nblk; u += gridDim.x) {
    const StreamSeg &sg = A.segs[find_seg(A.segs, A.nseg, u)];
    if (step_sweeps_of(A, sg.sys) != 1) continue;  // uniform per workgroup
    const SysDev &S = A.sysv[sg.sys];
    const int64_t local = (u - sg.blk0) * STREAM_BLOCK + threadIdx.x;
    if (local >= sg.count) continue;
    const int64_t b = local / S.N2;
    const int64_t r = local - b * S.N2;
    const int i = (int)(r / S.N);
    const int jj = (int)(r - (int64_t)i * S.N);
    const uint64_t di = A.desc[S.tab_off + i], dj = A.desc[S.tab_off + jj];
    const double gam = diag_rate(S, di, dj);
    const double dE = A.Etab[S.tab_off + i] - A.Etab[S.tab_off + jj];
    const int64_t e = sg.off + local;
    const double2 qv = A.q[e];
    step_output<ADJ>(A, e, S.h, diag_coef(gam, dE, ADJ), stage_weight(S.h, gam, dE, ADJ), qv,
                     csub(A.z0[e], qv));
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
    if (A.gpart && K < 2) K = 2;  // the integrands are formed in a sweep after the first
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
// Two-pass sweep and apply of one system (a state too large for the caches).
//
// The off-diagonal part is a sum over subsystems.  Pass A forms the terms of
// the subsystems q0..Q-1 (the least significant digits, level product NA)
// and pass B adds those of 0..q0-1 and finishes the entry.  Each pass works
// on sets of entries that contain all of its neighbours:
// * pass A: an NA x NA block of the state (the high row and column digits
//   fixed; rows and columns contiguous);
// * pass B: the entries with fixed low row digits and fixed low column
//   digits, except the SP lowest column values, which stay as contiguous
//   runs for coalescing (NB x NB x SP entries, NB = N / NA).
// Each workgroup takes 256 entries of one set and the sets are dealt to the
// XCDs in contiguous bands, so a set's neighbours are read from the L2 its
// own loads fill.  Pass A writes its partial sum to the output buffer of the
// sweep (or to y), where pass B reads it back entry by entry.
// ----------------------------------------------------------------------------
struct SplitPass {
  const SysDev *sysv;
  const uint64_t *desc;
  int sys, B, q0;
  int64_t NA, SP;
};

// Unit u of pass A (XCD band mapping applied by the caller) and thread tid:
// the entry, or false past the set's end.
__device__ __forceinline__ bool split_a_entry(const SplitPass &P, const SysDev &S, int64_t u, int tid, int64_t &b,
                                              int64_t &i, int64_t &j) {
  const int64_t NA = P.NA, NB = S.N / NA;
  const int64_t parts = (NA * NA + 255) / 256;
  const int64_t t = u / parts, f = (u - t * parts) * 256 + tid;
  if (f >= NA * NA) return false;
  b = t / (NB * NB);
  const int64_t rem = t - b * NB * NB;
  const int64_t hr = rem / NB, hc = rem - (rem / NB) * NB;
  const int64_t ar = f / NA, ac = f - (f / NA) * NA;
  i = hr * NA + ar;
  j = hc * NA + ac;
  return true;
}

__device__ __forceinline__ bool split_b_entry(const SplitPass &P, const SysDev &S, int64_t u, int tid, int64_t &b,
                                              int64_t &i, int64_t &j) {
  const int64_t NA = P.NA, NB = S.N / NA, SP = P.SP, NCB = NA / SP;
  const int64_t setsz = NB * NB * SP;
  const int64_t parts = (setsz + 255) / 256;
  const int64_t set = u / parts, f = (u - set * parts) * 256 + tid;
  if (f >= setsz) return false;
  b = set / (NA * NCB);
  const int64_t rem = set - b * NA * NCB;
  const int64_t rlo = rem / NCB, cb = rem - (rem / NCB) * NCB;
  const int64_t sp = f % SP, g = f / SP;
  const int64_t bc = g % NB, br = g / NB;
  i = br * NA + rlo;
  j = bc * NA + cb * SP + sp;
  return true;
}

__host__ __device__ inline int64_t split_units(int64_t N, int64_t NA, int64_t SP, int B, bool passA) {
  const int64_t NB = N / NA;
  if (passA) return (int64_t)B * NB * NB * ((NA * NA + 255) / 256);
  return (int64_t)B * NA * (NA / SP) * ((NB * NB * SP + 255) / 256);
}

__device__ __forceinline__ int64_t split_band(int64_t units) {
  const int64_t per = (units + 7) / 8;
  return (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Pass A: acc[e] = sum over q0 <= q < Q of the off-diagonal terms of x (M or
// M^+).  Controls: dtab[q] when given (a sweep: the step's row of the
// control table), else d_q(t) from alpha.  kstep: a sweep's count (launches
// at or past it return at once), or NULL.
template <bool ADJ>
__global__ __launch_bounds__(256) void split_a_kernel(SplitPass P, const double2 *__restrict__ dtab,
                                                      const double *__restrict__ alpha,
                                                      const double *__restrict__ carrier, double t,
                                                      const int32_t *__restrict__ kstep, int kk,
                                                      const double2 *__restrict__ x, double2 *__restrict__ acc) {
  if (kstep && kk > 0 && kk >= *kstep) return;  // uniform per launch
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dq[QMAX];
  const SysDev &S = P.sysv[P.sys];
  const int64_t units = split_units(S.N, P.NA, P.SP, P.B, true);
  const int64_t u = split_band(units);
  if (u >= units) return;  // uniform per workgroup
  const int tid = threadIdx.x;
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  if (tid < S.Q) dq[tid] = dtab ? dtab[tid] : control_value(S, alpha, carrier + S.carrier_off, tid, t);
  __syncthreads();
  int64_t b, i, j;
  if (!split_a_entry(P, S, u, tid, b, i, j)) return;
  const uint64_t di = P.desc[S.tab_off + i], dj = P.desc[S.tab_off + j];
  const double2 *xs = x + b * S.N2;
  const int64_t r = i * S.N + j;
  acc[b * S.N2 + r] =
      offdiag_range<ADJ>(S, di, dj, r, dq, sq, [&](int64_t idx) { return xs[idx]; }, P.q0, S.Q);
}

// Pass B of lindblad_apply: y = acc + (terms of q < q0) + D x.
template <bool ADJ>
__global__ __launch_bounds__(256) void split_b_apply_kernel(SplitPass P, const double *__restrict__ Etab,
                                                            const double *__restrict__ alpha,
                                                            const double *__restrict__ carrier, double t,
                                                            const double2 *__restrict__ x, double2 *__restrict__ y) {
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dq[QMAX];
  const SysDev &S = P.sysv[P.sys];
  const int64_t units = split_units(S.N, P.NA, P.SP, P.B, false);
  const int64_t u = split_band(units);
  if (u >= units) return;
  const int tid = threadIdx.x;
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  if (tid < S.Q) dq[tid] = control_value(S, alpha, carrier + S.carrier_off, tid, t);
  __syncthreads();
  int64_t b, i, j;
  if (!split_b_entry(P, S, u, tid, b, i, j)) return;
  const uint64_t di = P.desc[S.tab_off + i], dj = P.desc[S.tab_off + j];
  const double2 *xs = x + b * S.N2;
  const int64_t r = i * S.N + j, e = b * S.N2 + r;
  const double2 acc = cadd(y[e], offdiag_range<ADJ>(S, di, dj, r, dq, sq, [&](int64_t idx) { return xs[idx]; },
                                                    0, P.q0));
  const double gam = diag_rate(S, di, dj);
  const double dE = Etab[S.tab_off + i] - Etab[S.tab_off + j];
  y[e] = cadd(acc, cmul(diag_coef(gam, dE, ADJ), xs[r]));
}

// Pass B of stage sweep kk: the partial sum of pass A is in the sweep's
// output buffer (so.zo); the entry is finished like the other sweep kernels.
template <bool ADJ>
__global__ __launch_bounds__(256) void split_b_sweep_kernel(StepArgs A, int kk) {
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dq[QMAX];
  __shared__ double red[2][4];
  const SysDev &S = A.sysv[A.sys];
  int K = 2;
  if (kk > 0) {
    K = step_sweeps_of(A, A.sys);
    if (kk >= K) return;  // uniform per launch
  }
  const SplitPass P{A.sysv, A.desc, A.sys, A.B, A.split_q, A.split_na, A.split_sp};
  const int64_t units = split_units(S.N, P.NA, P.SP, P.B, false);
  const int64_t u = split_band(units);
  if (u >= units) return;  // uniform per workgroup
  const int tid = threadIdx.x;
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  if (tid < S.Q) dq[tid] = A.ctab[S.ctab_off + (int64_t)A.j * S.Q + tid - A.cshift];
  __syncthreads();
  SweepOut so;
  so.first = kk == 0;
  so.last = kk > 0 && kk == K - 1;
  so.zo = (kk & 1) ? A.z1 : A.z0;
  const double2 *zin = sweep_input(A, kk);
  int64_t b, i, j;
  if (split_b_entry(P, S, u, tid, b, i, j)) {
    const uint64_t di = A.desc[S.tab_off + i], dj = A.desc[S.tab_off + j];
    const double2 *zs = zin + b * S.N2;
    const int64_t r = i * S.N + j, e = b * S.N2 + r;
    const double2 acc = cadd(so.zo[e], offdiag_range<ADJ>(S, di, dj, r, dq, sq,
                                                          [&](int64_t idx) { return zs[idx]; }, 0, P.q0));
    sweep_entry<ADJ>(A, so, e, S.h, diag_rate(S, di, dj), A.Etab[S.tab_off + i] - A.Etab[S.tab_off + j], acc,
                     zs[r]);
  }
  if (so.first) {
    block_max2<256>(so.e1, so.qm, red);
    if (tid == 0) {
      unsigned long long *sl = slot_base(A, A.par, A.sys);
      atomicMax(&sl[blockIdx.x % LB_STEP_SLOTS], dbits(so.e1));
      atomicMax(&sl[LB_STEP_SLOTS + blockIdx.x % LB_STEP_SLOTS], dbits(so.qm));
    }
  }
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
  if (adj && A.gpart && kk > 0) {  // the step's last sweep with its gradient integrands
    // same blocks, twice the threads where a thread would hold more than 5 entries
    constexpr int GB = (Sh::EPT > 5 && BLOCK < 512) ? 2 * BLOCK : BLOCK;
    const void *g = (const void *)sweep_tile_grad_kernel<NL, QC, KR, KC, GB>;
    LBX_HIP(hipFuncSetAttribute(g, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(2 * shmem)));
    hipLaunchKernelGGL((sweep_tile_grad_kernel<NL, QC, KR, KC, GB>), grid, dim3(GB), 2 * shmem, st, A, kk);
    LBX_HIP(hipGetLastError());
  }
  return LB_OK;
}

}  // namespace

namespace {

int split_sweep_launch(const lb_plan *p, StepArgs &A, int kk, bool adj, const SplitGeo &g, hipStream_t st) {
  const SysDev &S = p->sys[A.sys];
  A.split_q = g.q0;
  A.split_na = g.NA;
  A.split_sp = g.SP;
  const SplitPass P{A.sysv, A.desc, A.sys, A.B, g.q0, g.NA, g.SP};
  const double2 *dtab = A.ctab + (S.ctab_off + (int64_t)A.j * S.Q - A.cshift);
  const int32_t *kst = A.kstep + (int64_t)A.par * A.nsys + A.sys;
  double2 *acc = (kk & 1) ? A.z1 : A.z0;
  const double2 *zin = sweep_input(A, kk);
  const int64_t ua = split_units(S.N, g.NA, g.SP, A.B, true), ub = split_units(S.N, g.NA, g.SP, A.B, false);
  const dim3 ga((unsigned)(((ua + 7) / 8) * 8)), gb((unsigned)(((ub + 7) / 8) * 8));
  if (adj) {
    hipLaunchKernelGGL(split_a_kernel<true>, ga, dim3(256), 0, st, P, dtab, nullptr, nullptr, 0.0, kst, kk, zin,
                       acc);
    hipLaunchKernelGGL(split_b_sweep_kernel<true>, gb, dim3(256), 0, st, A, kk);
  } else {
    hipLaunchKernelGGL(split_a_kernel<false>, ga, dim3(256), 0, st, P, dtab, nullptr, nullptr, 0.0, kst, kk, zin,
                       acc);
    hipLaunchKernelGGL(split_b_sweep_kernel<false>, gb, dim3(256), 0, st, A, kk);
  }
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

int sweep_only(const lb_plan *p, StepArgs &A, int kk, bool adj, int tile_sys, int tile_k, hipStream_t st) {
  if (tile_sys >= 0 && tile_k >= LB_SPLIT_BASE) {
    SplitGeo g;
    if (!split_geo(p, tile_sys, tile_k, &g)) return fail(LB_EUNSUPPORTED, "no two-pass split for this system");
    A.sys = tile_sys;
    return split_sweep_launch(p, A, kk, adj, g, st);
  }
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

bool split_geo(const lb_plan *p, int sys, int k, SplitGeo *g) {
  if (k < LB_SPLIT_BASE) return false;
  const SysDev &S = p->sys[sys];
  const int ka = k - LB_SPLIT_BASE;
  if (ka < 1 || ka >= S.Q || S.njc > 0) return false;
  g->q0 = S.Q - ka;
  g->NA = 1;
  for (int q = g->q0; q < S.Q; ++q) g->NA *= S.nlev[q];
  // spectator columns: the lowest column digits up to at least 8 values
  g->SP = 1;
  for (int q = S.Q - 1; q >= g->q0 && g->SP < 8; --q) g->SP *= S.nlev[q];
  return g->NA > 1 && S.N / g->NA > 1;
}

int launch_split_apply(const lb_plan *p, int sys, int B, bool adj, double t, const double *alpha,
                       const double2 *x, double2 *y, const SplitGeo &g, hipStream_t st) {
  if (B == 0) return LB_OK;
  const SysDev &S = p->sys[sys];
  const SplitPass P{p->d_sys, p->d_desc, sys, B, g.q0, g.NA, g.SP};
  const int64_t ua = split_units(S.N, g.NA, g.SP, B, true), ub = split_units(S.N, g.NA, g.SP, B, false);
  const dim3 ga((unsigned)(((ua + 7) / 8) * 8)), gb((unsigned)(((ub + 7) / 8) * 8));
  if (adj) {
    hipLaunchKernelGGL(split_a_kernel<true>, ga, dim3(256), 0, st, P, nullptr, alpha, p->d_carrier, t, nullptr, 0,
                       x, y);
    hipLaunchKernelGGL(split_b_apply_kernel<true>, gb, dim3(256), 0, st, P, p->d_E, alpha, p->d_carrier, t, x, y);
  } else {
    hipLaunchKernelGGL(split_a_kernel<false>, ga, dim3(256), 0, st, P, nullptr, alpha, p->d_carrier, t, nullptr, 0,
                       x, y);
    hipLaunchKernelGGL(split_b_apply_kernel<false>, gb, dim3(256), 0, st, P, p->d_E, alpha, p->d_carrier, t, x, y);
  }
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

namespace {

// Whether the fused last adjoint sweep of this block shape keeps every value
// in registers (no private memory): otherwise the separate integrand kernel
// is faster.
template <int NL, int QC, int KR, int KC, int BLOCK>
bool tile_grad_fused_fits() {
  using Sh = tile::Shape<NL, QC, KR, KC, BLOCK>;
  constexpr int GB = (Sh::EPT > 5 && BLOCK < 512) ? 2 * BLOCK : BLOCK;
  if (2 * Sh::lds_bytes() > (size_t)160 * 1024) return false;  // the block and the stage vector in LDS
  hipFuncAttributes fa{};
  if (hipFuncGetAttributes(&fa, (const void *)sweep_tile_grad_kernel<NL, QC, KR, KC, GB>) != hipSuccess) return false;
  return fa.localSizeBytes == 0;
}

}  // namespace

bool tile_grad_fusable(const lb_plan *p, int sys, int tile_k) {
  if (sys < 0 || tile_k <= 0 || tile_k >= LB_SPLIT_BASE) return false;
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0];
#define X(NL_, Q_, R_, C_, T_) \
  if (nl == NL_ && S.Q == Q_ && tile_k == 10 * R_ + C_) return tile_grad_fused_fits<NL_, Q_, R_, C_, T_>();
  LBX_TILE_SHAPES(X)
#undef X
  return false;
}

int launch_sweep(const lb_plan *p, StepArgs &A, int kk, bool adj, int tile_sys, int tile_k, hipStream_t st) {
  if (A.H > HMAX) return fail(LB_EINVAL, "increment history longer than the kernels keep");
  if (kk == 1 && !A.apriori && A.nblk > 0) {  // the steps whose first sweep sufficed
    const dim3 grid((unsigned)std::min<int64_t>(A.nblk, 2048));
    if (adj)
      hipLaunchKernelGGL(stage_finish_kernel<true>, grid, dim3(STREAM_BLOCK), 0, st, A);
    else
      hipLaunchKernelGGL(stage_finish_kernel<false>, grid, dim3(STREAM_BLOCK), 0, st, A);
    LBX_HIP(hipGetLastError());
  }
  if (int rc = sweep_only(p, A, kk, adj, tile_sys, tile_k, st)) return rc;
  if (kk == 0 && A.nseg > 0) {
    hipLaunchKernelGGL(step_count_kernel, dim3((unsigned)A.nseg), dim3(64), 0, st, A);
    LBX_HIP(hipGetLastError());
  }
  return LB_OK;
}

}  // namespace lbx
