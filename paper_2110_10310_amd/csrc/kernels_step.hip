// Persistent implicit-midpoint step kernels for streamed systems (states in
// HBM): one cooperative launch takes every stage-solve sweep of one step
// (App. A eqs. IMR and linsystem_primal; App. B eq. linsystem_adjoint for
// the adjoint), with grid-wide barriers between the sweeps.  The number of
// sweeps is decided on the device, a posteriori, so the host never needs it.
//
// Stage solve.  (I - h M) z = q with h = dt/2 and M = D + O is solved in
// delta form, z = q + delta:  delta <- w (h D q + h O (q + delta)),
// w = (1 - h D)^-1.  Since Re D <= 0, |w| <= 1 and the map contracts in the
// max norm with a factor theta_j <= h sum_q (2 |d_q| c_q + (n_q - 1)/T1_q)
// (control_table_kernel).  After a first sweep delta0 -> delta1 the error obeys
//   |delta1 - delta*| <= theta/(1 - theta) |delta1 - delta0|,
// and every further sweep multiplies the bound by theta; the kernel runs at
// least two sweeps and otherwise the fewest that bring the bound below
// tol * max|q|.  Both maxima are grid-wide: every workgroup writes its own
// partial maxima after the first sweep, and after the barrier every
// workgroup reduces all of them in the same order, so the count is the same
// in every workgroup (and every workgroup takes the same barriers).
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
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#include "lbx_host.hpp"
#include "tile_unit.hpp"

namespace lbx {

namespace {

namespace cg = cooperative_groups;

// Total sweeps of a stage solve after a first sweep that changed the iterate
// by e1 (max norm), with |q| <= qmax: at least two, at most kcap + 1.
__device__ __forceinline__ int stage_sweeps(double theta, double ratio, double e1, double qmax, double tol,
                                            int kcap, bool *capped) {
  double r = ratio * e1;
  const double lim = tol * qmax;
  int k = 0;
  while (r > lim && k < kcap) {
    r *= theta;
    ++k;
  }
  *capped = r > lim;
  return 1 + (k > 1 ? k : 1);
}

// Maximum over the workgroup (non-negative values), valid in thread 0.
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
  __syncthreads();
}

// Units of one launch dealt to workgroups: the workgroups of one XCD (they
// are dispatched to the 8 XCDs round-robin) walk a contiguous band of units.
struct Band {
  int64_t u0, u1, stride;
};
__device__ __forceinline__ Band xcd_band(int64_t units) {
  const int G = gridDim.x;  // a multiple of 8
  const int x = blockIdx.x & 7;
  const int64_t band = (units + 7) / 8;
  const int64_t lo = (int64_t)x * band;
  const int64_t hi = lo + band < units ? lo + band : units;
  return {lo + (blockIdx.x >> 3), hi, G / 8};
}

__device__ __forceinline__ double2 cfma(double2 acc, double c, double2 r, double2 d) {
  // acc + c * r * d
  const double2 rd = cmul(r, d);
  return make_double2(acc.x + c * rd.x, acc.y + c * rd.y);
}

// Start of the next step from the history (see the file comment): dn is this
// step's increment delta_n, R the diagonal Cayley factor, ring[k] holds
// delta_{n-k} for k = 1 .. m-1 at slot (n - k) mod H.
template <int HMAX>
__device__ __forceinline__ double2 next_start(double2 dn, double2 R, int m, int n, int H,
                                              const double2 *__restrict__ ring, int64_t stride, int64_t e) {
  // coefficients (-1)^k C(m, k+1)
  double2 Rk = R;
  double2 pred = make_double2(0.0, 0.0);
  double binom = (double)m;  // C(m, 1)
  pred = cfma(pred, binom, Rk, dn);
#pragma unroll
  for (int k = 1; k < HMAX; ++k) {
    if (k >= m) break;
    binom = binom * (double)(m - k) / (double)(k + 1);  // C(m, k+1)
    Rk = cmul(Rk, R);
    const int slot = ((n - k) % H + H) % H;
    const double2 d = ring[(int64_t)slot * stride + e];
    pred = cfma(pred, (k & 1) ? -binom : binom, Rk, d);
  }
  return pred;
}

constexpr int HMAX = 4;  // longest increment history

}  // namespace

// Status bits written by the kernels into the call's status word.
__device__ __forceinline__ void raise_status(int32_t *status, int bits) {
  if (status) atomicOr(status, bits);
}

// ----------------------------------------------------------------------------
// Block-tiled persistent step for one system of equal-level subsystems.
// ----------------------------------------------------------------------------
enum { SWEEP_FIRST = 1, SWEEP_LAST = 2 };

// One unit of one sweep.  Each unit builds its own stencil data (controls,
// subsystem tables, direction table), so nothing is hoisted across the
// persistent loop over units, whose live state would otherwise exceed the
// register file.  Returns the unit's maxima of |delta1 - delta0| and |q| on
// a first sweep.
template <int NL, int QC, int KR, int KC, bool ADJ, int BLOCK>
__device__ __forceinline__ double2 step_tile_unit(const SysDev *__restrict__ sysv, int sys, int64_t u, int j,
                                               const double2 *__restrict__ ctab, const double *__restrict__ Etab,
                                               const double2 *__restrict__ zin, const double2 *__restrict__ q,
                                               double2 *__restrict__ zo, double2 *__restrict__ out,
                                               double2 *__restrict__ zh, double2 *__restrict__ znext,
                                               double2 *__restrict__ ring, int64_t ring_stride, int n, int m,
                                               int H, int mode, bool again, double2 *tileb) {
  const SysDev &S = sysv[sys];
  const int lane = threadIdx.x & 63;
  const double h = S.h;
  double2 dv = make_double2(0.0, 0.0);
  if (lane < QC) dv = ctab[S.ctab_off + (int64_t)j * QC + lane];
  double da[QC], db[QC];
#pragma unroll
  for (int k = 0; k < QC; ++k) {
    da[k] = tile::lane_d(dv.x, k);
    db[k] = tile::lane_d(dv.y, k);
  }
  const bool first = mode & SWEEP_FIRST, last = mode & SWEEP_LAST;
  double e1 = 0.0, qm = 0.0;
  tile::tile_unit<NL, QC, KR, KC, ADJ, BLOCK>(S, u, zin, tileb, da, db, Etab + S.tab_off, again,
                                              [&](const tile::Entry &en) {
    const double2 qv = q[en.e];
    const double2 D = diag_coef(en.gam, en.dE, ADJ);
    const double2 w = stage_weight(h, en.gam, en.dE, ADJ);
    const double2 hdq = cscale(h, cmul(D, qv));
    const double2 dn = cmul(w, make_double2(hdq.x + h * en.acc.x, hdq.y + h * en.acc.y));
    if (first) {
      const double2 d0 = csub(en.own, qv);
      e1 = fmax(e1, fabs(dn.x - d0.x) + fabs(dn.y - d0.y));
      qm = fmax(qm, fmax(fabs(qv.x), fabs(qv.y)));
    }
    if (!last) {
      zo[en.e] = cadd(qv, dn);
      return;
    }
    const double2 qn = make_double2(qv.x + 2.0 * dn.x, qv.y + 2.0 * dn.y);
    out[en.e] = qn;
    if (ADJ && zh) zh[en.e] = cadd(qv, dn);
    if (znext) {
      const double2 R = cmul(make_double2(1.0 + h * D.x, h * D.y), w);
      const double2 pred = next_start<HMAX>(dn, R, m, n, H, ring, ring_stride, en.e);
      znext[en.e] = cadd(qn, pred);
      ring[(int64_t)(n % H) * ring_stride + en.e] = dn;
    }
  });
  return make_double2(e1, qm);
}

template <int NL, int QC, int KR, int KC, bool ADJ, int BLOCK>
__global__ __launch_bounds__(BLOCK) void step_tile_kernel(StepArgs A) {
  extern __shared__ double2 tileb[];
  __shared__ double red[2][BLOCK / 64];
  __shared__ int sK;
  cg::grid_group grid = cg::this_grid();
  const int tid = threadIdx.x;
  const Band bd = xcd_band(A.units);
  // Sweep kk reads zin (q + delta of sweep kk - 1; the start for kk = 0) and
  // writes z0 / z1 alternately; the count K is settled after sweep 0.
  int K = 2;
#pragma unroll 1
  for (int kk = 0; kk < K; ++kk) {
    const bool first = kk == 0, last = kk == K - 1;
    const double2 *zin = first ? (A.zstart ? A.zstart : A.q) : ((kk & 1) ? A.z0 : A.z1);
    double2 *zo = (kk & 1) ? A.z1 : A.z0;
    const int mode = (first ? SWEEP_FIRST : 0) | (last ? SWEEP_LAST : 0);
    double e1 = 0.0, qm = 0.0;
    bool again = false;
#pragma unroll 1
    for (int64_t u = bd.u0; u < bd.u1; u += bd.stride) {
      const double2 r = step_tile_unit<NL, QC, KR, KC, ADJ, BLOCK>(
          A.sysv, A.sys, u, A.j, A.ctab, A.Etab, zin, A.q, zo, A.out, A.zh, A.znext, A.ring, A.ring_stride, A.n,
          A.m, A.H, mode, again, tileb);
      e1 = fmax(e1, r.x);
      qm = fmax(qm, r.y);
      again = true;
    }
    if (first) {
      // sweep count from the grid-wide maxima, identical in every workgroup
      block_max2<BLOCK>(e1, qm, red);
      if (tid == 0) A.part[blockIdx.x] = make_double2(e1, qm);
      grid.sync();
      double ge = 0.0, gq = 0.0;
      for (int k = tid; k < (int)gridDim.x; k += BLOCK) {
        const double2 p = A.part[k];
        ge = fmax(ge, p.x);
        gq = fmax(gq, p.y);
      }
      block_max2<BLOCK>(ge, gq, red);
      if (tid == 0) {
        const double2 tt = A.ttab[(int64_t)A.sys * A.NT + A.j];
        bool capped = false;
        sK = stage_sweeps(tt.x, tt.y, ge, gq, A.tol, A.kcap, &capped);
        if (blockIdx.x == 0) {
          if (!(tt.x < 0.5)) raise_status(A.status, LB_STATUS_THETA);
          if (capped) raise_status(A.status, LB_STATUS_NOCONV);
          if (A.kout) A.kout[(int64_t)A.sys * A.NT + A.j] += sK;
        }
      }
      __syncthreads();
      K = sK;
    } else if (!last) {
      grid.sync();
    }
  }
}

// ----------------------------------------------------------------------------
// Generic persistent step over the segments of a streamed batch (any
// systems): one entry per thread, neighbours read directly from the batch.
// Every segment runs its own sweep count.
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
__global__ __launch_bounds__(STREAM_BLOCK) void step_generic_kernel(StepArgs A) {
  constexpr int BLOCK = STREAM_BLOCK;
  __shared__ double sq[SQRT_TABLE];
  __shared__ double red[2][BLOCK / 64];
  __shared__ int sK[LB_STEP_MAXSEG];
  __shared__ int sKmax;
  cg::grid_group grid = cg::this_grid();
  const int tid = threadIdx.x;
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);
  __syncthreads();
  const Band bd = xcd_band(A.nblk);
  // One unit = STREAM_BLOCK entries of one segment.  `body` forms delta at
  // this thread's entry of unit u with zin as the iterate.
  struct Loc {
    int seg;
    bool ok;
    int64_t e;  // entry in the compact streamed buffers
    double2 D, w;
    double2 dn;
    double2 qv;
    double2 own;
  };
  auto body = [&](int64_t u, const double2 *zin, Loc &L) {
    const int sgi = find_seg(A.segs, A.nseg, u);
    const StreamSeg &sg = A.segs[sgi];
    const SysDev &S = A.sysv[sg.sys];
    L.seg = sgi;
    const int64_t local = (u - sg.blk0) * BLOCK + tid;
    L.ok = local < sg.count;
    const int64_t lc = L.ok ? local : 0;
    const int64_t b = lc / S.N2;
    const int64_t r = lc - b * S.N2;
    const int i = (int)(r / S.N);
    const int jj = (int)(r - (int64_t)i * S.N);
    const uint64_t di = A.desc[S.tab_off + i], dj = A.desc[S.tab_off + jj];
    const double gam = diag_rate(S, di, dj);
    const double dE = A.Etab[S.tab_off + i] - A.Etab[S.tab_off + jj];
    double2 dq[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q)
      dq[q] = q < S.Q ? A.ctab[S.ctab_off + (int64_t)A.j * S.Q + q] : make_double2(0.0, 0.0);
    const int64_t base = sg.off + b * S.N2;
    L.e = base + r;
    L.D = diag_coef(gam, dE, ADJ);
    L.w = stage_weight(S.h, gam, dE, ADJ);
    const double2 acc = offdiag<ADJ>(S, di, dj, r, dq, sq, [&](int64_t idx) { return zin[base + idx]; });
    L.qv = A.q[L.e];
    L.own = zin[L.e];
    const double2 hdq = cscale(S.h, cmul(L.D, L.qv));
    L.dn = cmul(L.w, make_double2(hdq.x + S.h * acc.x, hdq.y + S.h * acc.y));
  };
  // Sweep kk reads zin and writes z0 / z1 alternately (see the tiled kernel);
  // the per-segment counts are settled after sweep 0.
  int Kmax = 2;
  for (int kk = 0; kk < Kmax; ++kk) {
    const bool first = kk == 0;
    const double2 *zin = first ? (A.zstart ? A.zstart : A.q) : ((kk & 1) ? A.z0 : A.z1);
    double2 *zo = (kk & 1) ? A.z1 : A.z0;
    for (int64_t u = bd.u0; u < bd.u1; u += bd.stride) {
      const int sgi = find_seg(A.segs, A.nseg, u);
      const int K = first ? 2 : sK[sgi];
      if (kk >= K) continue;  // uniform per unit
      const bool last = !first && kk == K - 1;
      Loc L;
      body(u, zin, L);
      double e1 = 0.0, qm = 0.0;
      if (L.ok) {
        if (first) {
          const double2 d0 = csub(L.own, L.qv);
          e1 = fabs(L.dn.x - d0.x) + fabs(L.dn.y - d0.y);
          qm = fmax(fabs(L.qv.x), fabs(L.qv.y));
        }
        if (!last) {
          zo[L.e] = cadd(L.qv, L.dn);
        } else {
          const SysDev &S = A.sysv[A.segs[sgi].sys];
          const double2 qn = make_double2(L.qv.x + 2.0 * L.dn.x, L.qv.y + 2.0 * L.dn.y);
          A.out[L.e] = qn;
          if (ADJ && A.zh) A.zh[L.e] = cadd(L.qv, L.dn);
          if (A.znext) {
            const double2 R = cmul(make_double2(1.0 + S.h * L.D.x, S.h * L.D.y), L.w);
            const double2 pred = next_start<HMAX>(L.dn, R, A.m, A.n, A.H, A.ring, A.ring_stride, L.e);
            A.znext[L.e] = cadd(qn, pred);
            A.ring[(int64_t)(A.n % A.H) * A.ring_stride + L.e] = L.dn;
          }
        }
      }
      if (first) {
        block_max2<BLOCK>(e1, qm, red);
        if (tid == 0) A.part[u] = make_double2(e1, qm);
      }
    }
    if (first) {
      grid.sync();
      // per-segment maxima: workgroup s reduces the units of segment s
      for (int s = blockIdx.x; s < A.nseg; s += gridDim.x) {
        const StreamSeg &sg = A.segs[s];
        const int64_t nu = (sg.count + BLOCK - 1) / BLOCK;
        double ge = 0.0, gq = 0.0;
        for (int64_t k = tid; k < nu; k += BLOCK) {
          const double2 p = A.part[sg.blk0 + k];
          ge = fmax(ge, p.x);
          gq = fmax(gq, p.y);
        }
        block_max2<BLOCK>(ge, gq, red);
        if (tid == 0) {
          const double2 tt = A.ttab[(int64_t)sg.sys * A.NT + A.j];
          bool capped = false;
          const int K = stage_sweeps(tt.x, tt.y, ge, gq, A.tol, A.kcap, &capped);
          A.segk[s] = K;
          if (!(tt.x < 0.5)) raise_status(A.status, LB_STATUS_THETA);
          if (capped) raise_status(A.status, LB_STATUS_NOCONV);
          if (A.kout) A.kout[(int64_t)sg.sys * A.NT + A.j] += K;
        }
      }
      grid.sync();
      if (tid == 0) sKmax = 0;
      __syncthreads();
      for (int s = tid; s < A.nseg; s += BLOCK) {
        const int K = A.segk[s];
        sK[s] = K;
        atomicMax(&sKmax, K);
      }
      __syncthreads();
      Kmax = sKmax;
    } else if (kk + 1 < Kmax) {
      grid.sync();
    }
  }
}

// ----------------------------------------------------------------------------
// Launchers
// ----------------------------------------------------------------------------
namespace {

struct CoopShape {
  int grid = 0;
  hipError_t err = hipSuccess;
};

// Workgroups of a cooperative launch: as many as can be resident at once
// (occupancy x compute units), a multiple of 8, at most `units` rounded up
// to a multiple of 8.
CoopShape coop_grid(const void *fn, int block, size_t shmem, int64_t units, int device) {
  static std::mutex mu;
  static std::map<std::tuple<const void *, int, size_t, int>, int> cache;
  int resident = 0;
  {
    std::lock_guard<std::mutex> g(mu);
    auto key = std::make_tuple(fn, block, shmem, device);
    auto it = cache.find(key);
    if (it != cache.end()) {
      resident = it->second;
    } else {
      int per_cu = 0, cus = 0;
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, shmem);
      if (e != hipSuccess) return {0, e};
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
      if (e != hipSuccess) return {0, e};
      resident = per_cu * cus;
      cache[key] = resident;
    }
  }
  int g = resident - resident % 8;
  const int64_t want = ((units + 7) / 8) * 8;
  if (want < g) g = (int)want;
  if (g < 8) return {0, hipErrorInvalidConfiguration};
  return {g, hipSuccess};
}

template <class F>
int coop_launch(F fn, int block, size_t shmem, int64_t units, int device, StepArgs &A, hipStream_t st,
                int *grid_out) {
  const void *f = (const void *)fn;
  if (shmem > 0) LBX_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const CoopShape cs = coop_grid(f, block, shmem, units, device);
  if (cs.err != hipSuccess) return hip_fail(cs.err, "cooperative grid size");
  if (grid_out) *grid_out = cs.grid;
  void *args[] = {&A};
  LBX_HIP(hipLaunchCooperativeKernel(f, dim3(cs.grid), dim3(block), args, (unsigned)shmem, st));
  return LB_OK;
}

template <int NL, int QC, int KR, int KC, int BLOCK>
int step_tile_launch(const lb_plan *p, StepArgs &A, bool adj, hipStream_t st, int *grid) {
  using Sh = tile::Shape<NL, QC, KR, KC, BLOCK>;
  A.units = tile::tile_units(p->sys[A.sys].N, Sh::TR, Sh::TC, A.B);
  if (adj)
    return coop_launch(step_tile_kernel<NL, QC, KR, KC, true, BLOCK>, BLOCK, Sh::lds_bytes(), A.units,
                       p->device, A, st, grid);
  return coop_launch(step_tile_kernel<NL, QC, KR, KC, false, BLOCK>, BLOCK, Sh::lds_bytes(), A.units,
                     p->device, A, st, grid);
}

}  // namespace

int launch_step(const lb_plan *p, StepArgs &A, bool adj, int tile_sys, int tile_k, hipStream_t st) {
  if (A.H > HMAX) return fail(LB_EINVAL, "increment history longer than the kernels keep");
  if (tile_sys >= 0) {
    const SysDev &S = p->sys[tile_sys];
    const int nl = S.nlev[0];
    A.sys = tile_sys;
#define X(NL_, Q_, R_, C_, T_)                                                    \
  if (nl == NL_ && S.Q == Q_ && tile_k == 10 * R_ + C_)                           \
    return step_tile_launch<NL_, Q_, R_, C_, T_>(p, A, adj, st, nullptr);
    LBX_TILE_SHAPES(X)
#undef X
    return fail(LB_EUNSUPPORTED, "no block-tiled step kernel for this system");
  }
  if (A.nseg > LB_STEP_MAXSEG) return fail(LB_EUNSUPPORTED, "too many streamed systems in one batch");
  if (adj)
    return coop_launch(step_generic_kernel<true>, STREAM_BLOCK, 0, A.nblk, p->device, A, st, nullptr);
  return coop_launch(step_generic_kernel<false>, STREAM_BLOCK, 0, A.nblk, p->device, A, st, nullptr);
}

// Grid (workgroups) the step kernels launch with: the size of the partial
// maxima array for the tiled kernels.
int step_grid(const lb_plan *p, int tile_sys, int tile_k, int B, int64_t nblk, int adj, int *grid) {
  *grid = 0;
  if (tile_sys >= 0) {
    const SysDev &S = p->sys[tile_sys];
    const int nl = S.nlev[0];
#define X(NL_, Q_, R_, C_, T_)                                                                        \
  if (nl == NL_ && S.Q == Q_ && tile_k == 10 * R_ + C_) {                                             \
    using Sh = tile::Shape<NL_, Q_, R_, C_, T_>;                                                      \
    const void *f = adj ? (const void *)step_tile_kernel<NL_, Q_, R_, C_, true, T_>                   \
                        : (const void *)step_tile_kernel<NL_, Q_, R_, C_, false, T_>;                 \
    LBX_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)Sh::lds_bytes())); \
    const CoopShape cs = coop_grid(f, T_, Sh::lds_bytes(), tile::tile_units(S.N, Sh::TR, Sh::TC, B),  \
                                   p->device);                                                        \
    if (cs.err != hipSuccess) return hip_fail(cs.err, "cooperative grid size");                       \
    *grid = cs.grid;                                                                                  \
    return LB_OK;                                                                                     \
  }
    LBX_TILE_SHAPES(X)
#undef X
    return fail(LB_EUNSUPPORTED, "no block-tiled step kernel for this system");
  }
  const void *f = adj ? (const void *)step_generic_kernel<true> : (const void *)step_generic_kernel<false>;
  const CoopShape cs = coop_grid(f, STREAM_BLOCK, 0, nblk, p->device);
  if (cs.err != hipSuccess) return hip_fail(cs.err, "cooperative grid size");
  *grid = cs.grid;
  return LB_OK;
}

}  // namespace lbx
