// LDS-resident persistent kernels specialised on the number of subsystems.
//
// Same memory layout as the generic kernels of kernels_lds.hip (one
// workgroup per state, stage iterate in two LDS buffers, delta-form
// fixed-point sweeps), for systems of one to four subsystems with one entry
// per thread.  Everything that does not change over the time loop is
// computed once per entry and kept in registers: the ladder weights sqrt(n),
// sqrt(n+1), sqrt(m), sqrt(m+1) with the boundary cases folded in as zeros,
// the decay-jump weight, and the LDS offsets of every neighbour (the entry
// itself where a neighbour does not exist, with a zero weight).  A sweep is
// then LDS reads and FP64 FMAs only.  Unlike the generic kernels they start
// each stage solve from an extrapolation of earlier steps and stop on an
// a-posteriori bound (see extra_sweeps); the per-step controls come through a
// vector load one step ahead.  The adjoint stores each step's stage vector,
// and lds_grad_fast_kernel forms the gradient integrands of all steps after
// it, reduced over 16-lane DPP rows.
#include <hip/hip_runtime.h>

#include "lbx_host.hpp"

namespace lbx {

namespace {

template <int CTRL>
__device__ __forceinline__ double dpp_row_shift(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Inclusive prefix sum within each row of 16 lanes: lane 15 of a row holds
// the sum of the row (fixed order, hence deterministic).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_row_shift<0x111>(v);
  v += dpp_row_shift<0x112>(v);
  v += dpp_row_shift<0x114>(v);
  v += dpp_row_shift<0x118>(v);
  return v;
}

// Per-(entry, subsystem) stencil data, fixed for the whole time loop.
struct Nb {
  double crp, crm, ccp, ccm, cj;  // weights of rows +/-, columns +/-, jump
  int orp, orm, ocp, ocm, oj;     // LDS offsets of those neighbours
};

template <bool ADJ>
__device__ __forceinline__ Nb make_nb(const SysDev &S, int q, uint64_t di, uint64_t dj, int e) {
  Nb b;
  const int n = digit(di, q), m = digit(dj, q);
  const int nl = S.nlev[q];
  const int s1 = S.stride[q];
  const int sN = s1 * S.N;
  const bool rp = n + 1 < nl, rm = n > 0, cp = m + 1 < nl, cm = m > 0;
  b.crp = rp ? sqrt((double)(n + 1)) : 0.0;
  b.crm = sqrt((double)n);
  b.ccp = cp ? sqrt((double)(m + 1)) : 0.0;
  b.ccm = sqrt((double)m);
  b.orp = rp ? e + sN : e;
  b.orm = rm ? e - sN : e;
  b.ocp = cp ? e + s1 : e;
  b.ocm = cm ? e - s1 : e;
  if (!ADJ) {
    const bool ok = rp && cp;
    b.cj = ok ? S.g1[q] * sqrt((double)((n + 1) * (m + 1))) : 0.0;
    b.oj = ok ? e + sN + s1 : e;
  } else {
    const bool ok = rm && cm;
    b.cj = ok ? S.g1[q] * sqrt((double)(n * m)) : 0.0;
    b.oj = ok ? e - sN - s1 : e;
  }
  return b;
}

// U = sqrt(n+1) x_{i+e,j} - sqrt(m) x_{i,j-e},  V = sqrt(n) x_{i-e,j} - sqrt(m+1) x_{i,j+e}.
__device__ __forceinline__ void uv(const Nb &b, const double2 *x, double2 &U, double2 &V) {
  const double2 xrp = x[b.orp], xrm = x[b.orm], xcp = x[b.ocp], xcm = x[b.ocm];
  U = make_double2(b.crp * xrp.x - b.ccm * xcm.x, b.crp * xrp.y - b.ccm * xcm.y);
  V = make_double2(b.crm * xrm.x - b.ccp * xcp.x, b.crm * xrm.y - b.ccp * xcp.y);
}

// O x (forward) or O^+ x (adjoint) at one entry; see `offdiag` in lbx_device.hpp.
template <bool ADJ, int QC>
__device__ __forceinline__ double2 offdiag_nb(const Nb (&nb)[QC], const double2 (&dq)[QC],
                                              const double2 *x) {
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    double2 U, V;
    uv(nb[q], x, U, V);
    const double2 Sm = cadd(U, V), Dv = csub(U, V);
    const double a = dq[q].x, b = dq[q].y;
    const double cr = a * Sm.y + b * Dv.x;
    const double ci = -a * Sm.x + b * Dv.y;
    const double2 xj = x[nb[q].oj];
    if (!ADJ) {
      acc.x += cr + nb[q].cj * xj.x;
      acc.y += ci + nb[q].cj * xj.y;
    } else {
      acc.x += -cr + nb[q].cj * xj.x;
      acc.y += -ci + nb[q].cj * xj.y;
    }
  }
  return acc;
}

}  // namespace

// Stage solve with an extrapolated start and an a-posteriori sweep count.
//
// The fixed-point map delta -> w (h D q + h O (q + delta)) contracts in the
// max norm with factor theta (see control_table_kernel), so after a first
// sweep delta0 -> delta1 the error obeys |delta1 - delta*| <= theta/(1 - theta)
// |delta1 - delta0|, and every further sweep multiplies that bound by theta.
// The kernels start from the polynomial extrapolation of the last converged
// deltas (the stage increment varies smoothly with t), measure
// |delta1 - delta0| and max|q| once per step over the workgroup, and run at
// least two sweeps and otherwise the smallest number that brings the bound
// below tol max|q|.  Every thread reads the same two maxima from LDS, so the
// count is uniform.
__device__ __forceinline__ int extra_sweeps(double theta, double ratio, double e1, double qmax,
                                            double tol, int32_t *status) {
  double r = ratio * e1;  // ratio = theta / (1 - theta), from the control table
  const double lim = tol * qmax;
  int k = 0;
  // The usual counts without branches (so the compiler can interleave them
  // with the second sweep), then a loop for the rare remainder.
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const bool more = r > lim;
    k += more ? 1 : 0;
    r = more ? r * theta : r;
  }
  while (r > lim && k < 64) {
    r *= theta;
    ++k;
  }
  // A step whose contraction bound is >= 0.5, or that the cap stops, is
  // reported through the status word (LB_STATUS_*).
  if (status && threadIdx.x == 0 && (!(theta < 0.5) || r > lim))
    atomicOr(status, !(theta < 0.5) ? LB_STATUS_THETA : LB_STATUS_NOCONV);
  return k;
}

// Start of the stage iteration at step number `n` of the sweep direction:
// w h D q at the first step, then the polynomial extrapolation of the
// previous converged deltas d[0] (latest) .. d[H-1] of the highest order
// they allow, up to H - 1 (the controls are piecewise quadratic in t, so
// delta is smooth between B-spline knots).
template <int H>
__device__ __forceinline__ double2 extrapolated_start(int n, double2 w, double2 hdq,
                                                      const double2 (&d)[H]) {
  static_assert(H >= 2 && H <= 6, "history of 2 to 6 deltas");
  if (n == 0) return cmul(w, hdq);
  // coefficients (-1)^i C(m, i+1) of the order-(m-1) extrapolation, m = min(n, H)
  const int m = n < H ? n : H;
  const double c0 = (double)m;
  const double c1 = m >= 2 ? -(double)(m * (m - 1) / 2) : 0.0;
  double2 r = make_double2(c0 * d[0].x + c1 * d[1].x, c0 * d[0].y + c1 * d[1].y);
  if constexpr (H >= 3) {
    const double c2 = m >= 3 ? (double)(m * (m - 1) * (m - 2) / 6) : 0.0;
    r.x += c2 * d[2].x;
    r.y += c2 * d[2].y;
  }
  if constexpr (H >= 4) {
    const double c3 = m >= 4 ? -(double)(m * (m - 1) * (m - 2) * (m - 3) / 24) : 0.0;
    r.x += c3 * d[3].x;
    r.y += c3 * d[3].y;
  }
  if constexpr (H >= 5) {
    const double c4 = m >= 5 ? (double)(m * (m - 1) * (m - 2) * (m - 3) * (m - 4) / 120) : 0.0;
    r.x += c4 * d[4].x;
    r.y += c4 * d[4].y;
  }
  if constexpr (H >= 6) {
    const double c5 = m >= 6 ? -1.0 : 0.0;
    r.x += c5 * d[5].x;
    r.y += c5 * d[5].y;
  }
  return r;
}

// Deltas kept for the extrapolation: six (order 5) except on 1024-thread
// workgroups (one subsystem only, see lds_fast_ok), order 2.
template <int BLOCK>
constexpr int hist_len() { return BLOCK >= 1024 ? 3 : 6; }

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Maximum over the wavefront of 32-bit unsigned values: prefix maxima within
// rows of 16 lanes, then the four row maxima.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_row_shift_u(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, dpp_row_shift_u<0x111>(v));
  v = max(v, dpp_row_shift_u<0x112>(v));
  v = max(v, dpp_row_shift_u<0x114>(v));
  v = max(v, dpp_row_shift_u<0x118>(v));
  const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
  const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
  const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
  const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
  return max(max(a, b), max(c, d));
}

// The block maxima of the first-sweep change and of |q| are reduced on the
// high words of the (non-negative) doubles, which order like the values:
// the change is then bounded from above (low word all ones) and max|q| from
// below (low word zero), both within a relative 2^-20.
__device__ __forceinline__ double hi_upper(uint32_t hi) { return __hiloint2double((int)hi, -1); }
__device__ __forceinline__ double hi_lower(uint32_t hi) { return __hiloint2double((int)hi, 0); }

// Per-step constants of step j, one double per lane: the controls d_q in
// lanes 0 .. 2 QC - 1, then theta and theta / (1 - theta).  A vector load, so
// that the load for the next step is in flight during this one.
struct StepConst {
  double theta, ratio;
};

template <int QC>
__device__ __forceinline__ double load_controls(const double2 *cq, const double2 *tq, int j, int NT,
                                                int lane) {
  const int jj = j < NT ? j : NT - 1;
  const double *c = (const double *)(cq + (int64_t)jj * QC);
  const double *t = (const double *)(tq + jj);
  return lane < 2 * QC ? c[lane] : t[lane == 2 * QC ? 0 : 1];
}

template <int QC>
__device__ __forceinline__ StepConst unpack_controls(double v, double2 (&dq)[QC]) {
#pragma unroll
  for (int q = 0; q < QC; ++q) dq[q] = make_double2(readlane_d(v, 2 * q), readlane_d(v, 2 * q + 1));
  return {readlane_d(v, 2 * QC), readlane_d(v, 2 * QC + 1)};
}

template <int BLOCK, int EPT, int QC>
__global__ __launch_bounds__(BLOCK) void lds_forward_fast_kernel(
    const SysDev *__restrict__ sysv, const LdsItem *__restrict__ items,
    const double *__restrict__ Etab, const uint64_t *__restrict__ desc,
    const double2 *__restrict__ ctab, const double2 *__restrict__ ttab, double tol, int NT,
    const double2 *__restrict__ rho0, double2 *__restrict__ rhoT, double2 *__restrict__ states,
    int64_t *__restrict__ sweeps, int32_t *__restrict__ status) {
  extern __shared__ double2 zbuf[];
  constexpr int WAVES = BLOCK / 64;
  __shared__ uint32_t wmax[2][WAVES];
  const LdsItem it = items[blockIdx.x];
  const SysDev &S = sysv[it.sys];
  const int tid = threadIdx.x, lane = tid & 63;
  const int N = S.N;
  const int N2 = (int)S.N2;
  const double h = S.h;
  const double2 *cq = ctab + S.ctab_off;

  constexpr int HL = hist_len<BLOCK>();
  double2 qv[EPT], wv[EPT], hd[EPT], dn[EPT], dh[EPT][HL];
  Nb nb[EPT][QC];
  int ee[EPT];
  bool ok[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * BLOCK;
    ok[k] = e < N2;
    ee[k] = ok[k] ? e : 0;
    const int i = ee[k] / N, jj = ee[k] - (ee[k] / N) * N;
    const uint64_t di = desc[S.tab_off + i], dj = desc[S.tab_off + jj];
    const double gam = diag_rate(S, di, dj);
    const double dE = Etab[S.tab_off + i] - Etab[S.tab_off + jj];
    wv[k] = stage_weight(h, gam, dE, false);
    hd[k] = cscale(h, diag_coef(gam, dE, false));
#pragma unroll
    for (int q = 0; q < QC; ++q) nb[k][q] = make_nb<false>(S, q, di, dj, ee[k]);
    qv[k] = ok[k] ? rho0[it.off + e] : make_double2(0.0, 0.0);
    dn[k] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < HL; ++i) dh[k][i] = make_double2(0.0, 0.0);
    if (states && ok[k]) states[it.st_off + e] = qv[k];
  }
  // Two LDS stage buffers; selected by value (not through a pointer array)
  // so that every access stays an LDS instruction.
  double2 *const zb0 = zbuf, *const zb1 = zbuf + N2;
  int cb = 0;
  int64_t nsw = 0;
  // Controls of step j + 1 are loaded during step j and unpacked before
  // the state store of step j, so that waiting for them never waits for a
  // store just issued.
  const double2 *tq = ttab + (int64_t)it.sys * NT;
  double2 dq[QC];
  StepConst sc = unpack_controls<QC>(load_controls<QC>(cq, tq, 0, NT, lane), dq);
  double cnext = load_controls<QC>(cq, tq, 1, NT, lane);
  for (int j = 0; j < NT; ++j) {
    double2 hdq[EPT], d0[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      hdq[k] = cmul(hd[k], qv[k]);
      d0[k] = extrapolated_start(j, wv[k], hdq[k], dh[k]);
      if (ok[k]) (cb ? zb1 : zb0)[ee[k]] = cadd(qv[k], d0[k]);
    }
    __syncthreads();
    // first sweep, with the change it makes and max|q|
    double e1 = 0.0, qm = 0.0;
    {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<false, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
        if (ok[k]) {
          e1 = fmax(e1, fabs(dn[k].x - d0[k].x) + fabs(dn[k].y - d0[k].y));
          qm = fmax(qm, fmax(fabs(qv[k].x), fabs(qv[k].y)));
        }
      }
      const uint32_t he = wave_max_u32((uint32_t)__double2hiint(e1));
      const uint32_t hq = wave_max_u32((uint32_t)__double2hiint(qm));
      if (lane == 0) {
        wmax[0][tid >> 6] = he;
        wmax[1][tid >> 6] = hq;
      }
      double2 *dst = (cb ? zb0 : zb1);
#pragma unroll
      for (int k = 0; k < EPT; ++k)
        if (ok[k]) dst[ee[k]] = cadd(qv[k], dn[k]);
      __syncthreads();
      cb ^= 1;
    }
    // The second sweep runs in any case; the count of further ones is
    // settled while its LDS reads are in flight.
    {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<false, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
      }
    }
    uint32_t he = wmax[0][0], hq = wmax[1][0];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) {
      he = max(he, wmax[0][w]);
      hq = max(hq, wmax[1][w]);
    }
    const int K = extra_sweeps(sc.theta, sc.ratio, hi_upper(he), hi_lower(hq), tol, status);
    const int rest = K > 1 ? K - 1 : 0;
    nsw += 2 + rest;
    // Further sweeps: the iterate for the third is written (and the barrier
    // taken) before the count is known, so that the count's latency is
    // hidden; it is unused when two sweeps suffice.  The usual counts are
    // straight-line code.
    auto sweep_more = [&]() {
      double2 *dst = (cb ? zb0 : zb1);
#pragma unroll
      for (int k = 0; k < EPT; ++k)
        if (ok[k]) dst[ee[k]] = cadd(qv[k], dn[k]);
      __syncthreads();
      cb ^= 1;
    };
    auto sweep_math = [&]() {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<false, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
      }
    };
    sweep_more();
    if (rest >= 1) {
      sweep_math();
      if (rest >= 2) {
        sweep_more();
        sweep_math();
        for (int kk = 2; kk < rest; ++kk) {
          sweep_more();
          sweep_math();
        }
      }
    }
    sc = unpack_controls<QC>(cnext, dq);
    cnext = load_controls<QC>(cq, tq, j + 2, NT, lane);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      qv[k] = make_double2(qv[k].x + 2.0 * dn[k].x, qv[k].y + 2.0 * dn[k].y);
#pragma unroll
      for (int i = HL - 1; i > 0; --i) dh[k][i] = dh[k][i - 1];
      dh[k][0] = dn[k];
      if (states && ok[k]) states[it.st_off + (int64_t)(j + 1) * N2 + ee[k]] = qv[k];
    }
    cb ^= 1;
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k)
    if (ok[k]) rhoT[it.off + ee[k]] = qv[k];
  if (sweeps && tid == 0) sweeps[blockIdx.x] = nsw;
}

template <int BLOCK, int EPT, int QC>
__global__ __launch_bounds__(BLOCK) void lds_adjoint_fast_kernel(
    const SysDev *__restrict__ sysv, const LdsItem *__restrict__ items,
    const double *__restrict__ Etab, const uint64_t *__restrict__ desc,
    const double2 *__restrict__ ctab, const double2 *__restrict__ ttab, double tol, int NT,
    int kind, const double2 *__restrict__ rhotar, const double2 *__restrict__ states,
    double2 *__restrict__ zhist, int64_t *__restrict__ sweeps, int32_t *__restrict__ status) {
  extern __shared__ double2 zbuf[];
  constexpr int WAVES = BLOCK / 64;
  __shared__ uint32_t wmax[2][WAVES];
  const LdsItem it = items[blockIdx.x];
  const SysDev &S = sysv[it.sys];
  const int tid = threadIdx.x, lane = tid & 63;
  const int N = S.N;
  const int N2 = (int)S.N2;
  const double h = S.h;
  const double2 *cq = ctab + S.ctab_off;
  const double2 *hist = states + it.st_off;

  constexpr int HL = hist_len<BLOCK>();
  double2 qh[EPT], wv[EPT], hd[EPT], dn[EPT], dh[EPT][HL];
  Nb nb[EPT][QC];
  int ee[EPT];
  bool ok[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * BLOCK;
    ok[k] = e < N2;
    ee[k] = ok[k] ? e : 0;
    const int i = ee[k] / N, jj = ee[k] - (ee[k] / N) * N;
    const uint64_t di = desc[S.tab_off + i], dj = desc[S.tab_off + jj];
    const double gam = diag_rate(S, di, dj);
    const double dE = Etab[S.tab_off + i] - Etab[S.tab_off + jj];
    wv[k] = stage_weight(h, gam, dE, true);
    hd[k] = cscale(h, diag_coef(gam, dE, true));
#pragma unroll
    for (int q = 0; q < QC; ++q) nb[k][q] = make_nb<true>(S, q, di, dj, ee[k]);
    // Terminal condition (App. B): qh = (beta/M) dJ/d(conj q) at q = rho(T).
    const double2 qT = ok[k] ? hist[(int64_t)NT * N2 + ee[k]] : make_double2(0.0, 0.0);
    const double2 t = ok[k] ? rhotar[it.off + ee[k]] : make_double2(0.0, 0.0);
    qh[k] = kind == LB_J_FROB ? cscale(it.wterm, csub(qT, t)) : cscale(kind == LB_J_NM ? it.wterm : -it.wterm, t);
    dn[k] = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < HL; ++i) dh[k][i] = make_double2(0.0, 0.0);
  }
  double2 *const zb0 = zbuf, *const zb1 = zbuf + N2;
  int cb = 0;
  int64_t nsw = 0;
  // Controls of step j - 1 are loaded at the top of step j and unpacked after
  // its sweeps.
  const double2 *tq = ttab + (int64_t)it.sys * NT;
  double2 dq[QC];
  StepConst sc = unpack_controls<QC>(load_controls<QC>(cq, tq, NT - 1, NT, lane), dq);
  for (int j = NT - 1; j >= 0; --j) {
    const double cnext = load_controls<QC>(cq, tq, j > 0 ? j - 1 : 0, NT, lane);
    // (I - h M^+) zh = qh^{j+1} (App. B eq. linsystem_adjoint), zh = qh + delta.
    double2 hdq[EPT], d0[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      hdq[k] = cmul(hd[k], qh[k]);
      d0[k] = extrapolated_start(NT - 1 - j, wv[k], hdq[k], dh[k]);
      if (ok[k]) (cb ? zb1 : zb0)[ee[k]] = cadd(qh[k], d0[k]);
    }
    __syncthreads();
    double e1 = 0.0, qm = 0.0;
    {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<true, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
        if (ok[k]) {
          e1 = fmax(e1, fabs(dn[k].x - d0[k].x) + fabs(dn[k].y - d0[k].y));
          qm = fmax(qm, fmax(fabs(qh[k].x), fabs(qh[k].y)));
        }
      }
      const uint32_t he = wave_max_u32((uint32_t)__double2hiint(e1));
      const uint32_t hq = wave_max_u32((uint32_t)__double2hiint(qm));
      if (lane == 0) {
        wmax[0][tid >> 6] = he;
        wmax[1][tid >> 6] = hq;
      }
      double2 *dst = (cb ? zb0 : zb1);
#pragma unroll
      for (int k = 0; k < EPT; ++k)
        if (ok[k]) dst[ee[k]] = cadd(qh[k], dn[k]);
      __syncthreads();
      cb ^= 1;
    }
    // The second sweep runs in any case; the count of further ones is
    // settled while its LDS reads are in flight.
    {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<true, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
      }
    }
    uint32_t he = wmax[0][0], hq = wmax[1][0];
#pragma unroll
    for (int w = 1; w < WAVES; ++w) {
      he = max(he, wmax[0][w]);
      hq = max(hq, wmax[1][w]);
    }
    const int K = extra_sweeps(sc.theta, sc.ratio, hi_upper(he), hi_lower(hq), tol, status);
    const int rest = K > 1 ? K - 1 : 0;
    nsw += 2 + rest;
    // Further sweeps: the iterate for the third is written (and the barrier
    // taken) before the count is known, so that the count's latency is
    // hidden; it is unused when two sweeps suffice.  The usual counts are
    // straight-line code.
    auto sweep_more = [&]() {
      double2 *dst = (cb ? zb0 : zb1);
#pragma unroll
      for (int k = 0; k < EPT; ++k)
        if (ok[k]) dst[ee[k]] = cadd(qh[k], dn[k]);
      __syncthreads();
      cb ^= 1;
    };
    auto sweep_math = [&]() {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<true, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
      }
    };
    sweep_more();
    if (rest >= 1) {
      sweep_math();
      if (rest >= 2) {
        sweep_more();
        sweep_math();
        for (int kk = 2; kk < rest; ++kk) {
          sweep_more();
          sweep_math();
        }
      }
    }
    // The converged stage vector zh goes to HBM for the gradient integrands
    // (lds_grad_fast_kernel, after this loop), which leaves them off the
    // chain of dependent steps.
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      if (ok[k]) zhist[it.st_off + (int64_t)j * N2 + ee[k]] = cadd(qh[k], dn[k]);
    sc = unpack_controls<QC>(cnext, dq);
    // qh^j = qh^{j+1} + dt M^+ zh = qh^{j+1} + 2 delta.
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      qh[k] = make_double2(qh[k].x + 2.0 * dn[k].x, qh[k].y + 2.0 * dn[k].y);
#pragma unroll
      for (int i = HL - 1; i > 0; --i) dh[k][i] = dh[k][i - 1];
      dh[k][0] = dn[k];
    }
    // The next step's first iterate goes to the buffer the last sweep did not
    // read (all reads of the other one precede the last barrier).
    cb ^= 1;
  }
  if (sweeps && tid == 0) sweeps[blockIdx.x] = nsw;
}

// Gradient integrands of the specialised adjoint (App. B eq. reducedgradient,
// see grad_term in lbx_device.hpp), for all steps at once: workgroup (c, item)
// takes steps [c GCHUNK, (c + 1) GCHUNK) of one item.  Per step, zh^j is
// staged in LDS (two buffers by step parity, one barrier per step), z^j =
// (q^j + q^{j+1})/2 comes from the forward history, and each row of 16 lanes
// writes its partial sums, in the same order and layout as the integrands
// formed inside the adjoint loop would be.
constexpr int GCHUNK = 64;

template <int BLOCK, int QC>
__global__ __launch_bounds__(BLOCK) void lds_grad_fast_kernel(
    const SysDev *__restrict__ sysv, const LdsItem *__restrict__ items,
    const uint64_t *__restrict__ desc, int NT, const double2 *__restrict__ states,
    const double2 *__restrict__ zhist, double *__restrict__ gpart) {
  extern __shared__ double2 zbuf[];
  constexpr int ROWS = BLOCK / 16;
  const LdsItem it = items[blockIdx.y];
  const SysDev &S = sysv[it.sys];
  const int tid = threadIdx.x;
  const int N = S.N;
  const int N2 = (int)S.N2;
  const bool ok = tid < N2;
  const int e = ok ? tid : 0;
  const int i = e / N, jj = e - (e / N) * N;
  Nb nb[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) nb[q] = make_nb<true>(S, q, desc[S.tab_off + i], desc[S.tab_off + jj], e);
  const double2 *hist = states + it.st_off;
  const double2 *zh = zhist + it.st_off;
  const int j0 = (int)blockIdx.x * GCHUNK;
  const int j1 = min(NT, j0 + GCHUNK);
  for (int j = j0; j < j1; ++j) {
    double2 *zb = zbuf + (j & 1) * N2;
    if (ok) zb[e] = zh[(int64_t)j * N2 + e];
    const double2 qj = ok ? hist[(int64_t)j * N2 + e] : make_double2(0.0, 0.0);
    const double2 qn = ok ? hist[(int64_t)(j + 1) * N2 + e] : make_double2(0.0, 0.0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      double gp = 0.0, gq = 0.0;
      if (ok) {
        const double2 z = make_double2(0.5 * (qj.x + qn.x), 0.5 * (qj.y + qn.y));
        double2 U, V;
        uv(nb[q], zb, U, V);
        const double2 Sm = cadd(U, V), Dv = csub(U, V);
        gp += Sm.x * z.y - Sm.y * z.x;
        gq -= Dv.x * z.x + Dv.y * z.y;
      }
      gp = row16_sum(gp);
      gq = row16_sum(gq);
      if ((tid & 15) == 15) {
        double *dstp = gpart + it.gp_off + ((int64_t)j * ROWS + (tid >> 4)) * 2 * QC + 2 * q;
        dstp[0] = gp;
        dstp[1] = gq;
      }
    }
  }
}

// Shapes with a specialised kernel: one entry per thread.  Workgroups of
// 1024 threads leave 128 VGPRs per thread, which holds the register-resident
// stencil data of one subsystem only; larger ones use the generic kernels.
bool lds_fast_ok(int block, int ept, int Q) {
  if (Q < 1 || Q > 4 || ept != 1) return false;
  return block <= 512 || Q == 1;
}

template <int BLOCK, int EPT, int QC>
static int fwd_t(const lb_plan *p, const LdsItem *d_items, int nitems, const double2 *ctab,
                 const double2 *ttab, double tol, const double2 *rho0, double2 *rhoT, double2 *states,
                 int64_t *sweeps, int32_t *status, hipStream_t st) {
  const size_t shmem = (size_t)2 * BLOCK * EPT * sizeof(double2);
  auto kern = lds_forward_fast_kernel<BLOCK, EPT, QC>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(BLOCK), shmem, st, p->d_sys, d_items, p->d_E, p->d_desc,
                     ctab, ttab, tol, p->NT, rho0, rhoT, states, sweeps, status);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

template <int BLOCK, int EPT, int QC>
static int adj_t(const lb_plan *p, const LdsItem *d_items, int nitems, int kind, const double2 *ctab,
                 const double2 *ttab, double tol, const double2 *rhotar, const double2 *states,
                 double2 *zhist, double *gpart, int64_t *sweeps, int32_t *status, hipStream_t st) {
  const size_t shmem = (size_t)2 * BLOCK * EPT * sizeof(double2);
  auto kern = lds_adjoint_fast_kernel<BLOCK, EPT, QC>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(BLOCK), shmem, st, p->d_sys, d_items, p->d_E, p->d_desc,
                     ctab, ttab, tol, p->NT, kind, rhotar, states, zhist, sweeps, status);
  LBX_HIP(hipGetLastError());
  static_assert(EPT == 1, "the integrand kernel takes one entry per thread");
  auto gk = lds_grad_fast_kernel<BLOCK, QC>;
  LBX_HIP(hipFuncSetAttribute((const void *)gk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(gk, dim3((p->NT + GCHUNK - 1) / GCHUNK, nitems), dim3(BLOCK), shmem, st, p->d_sys,
                     d_items, p->d_desc, p->NT, states, zhist, gpart);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

#define LBX_FAST_SHAPES(X)                                                                  \
  X(64, 1, 1) X(64, 1, 2) X(64, 1, 3) X(64, 1, 4) X(128, 1, 1) X(128, 1, 2) X(128, 1, 3)    \
  X(128, 1, 4) X(256, 1, 1) X(256, 1, 2) X(256, 1, 3) X(256, 1, 4) X(512, 1, 1) X(512, 1, 2) \
  X(512, 1, 3) X(512, 1, 4) X(1024, 1, 1)

int launch_lds_forward_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, const double2 *ctab, const double2 *ttab, double tol, const double2 *rho0,
                            double2 *rhoT, double2 *states, int64_t *sweeps, int32_t *status, hipStream_t st) {
  if (nitems == 0) return LB_OK;
#define X(B, E, C) \
  if (block == B && ept == E && Q == C) return fwd_t<B, E, C>(p, d_items, nitems, ctab, ttab, tol, rho0, rhoT, states, sweeps, status, st);
  LBX_FAST_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "no specialised LDS-resident kernel for this shape");
}

int launch_lds_adjoint_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, int kind, const double2 *ctab, const double2 *ttab, double tol,
                            const double2 *rhotar, const double2 *states, double2 *zhist,
                            double *gpart, int64_t *sweeps, int32_t *status, hipStream_t st) {
  if (nitems == 0) return LB_OK;
  if (nitems > 65535) return fail(LB_EUNSUPPORTED, "more than 65535 states in one LDS kernel class");
#define X(B, E, C) \
  if (block == B && ept == E && Q == C) return adj_t<B, E, C>(p, d_items, nitems, kind, ctab, ttab, tol, rhotar, states, zhist, gpart, sweeps, status, st);
  LBX_FAST_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "no specialised LDS-resident kernel for this shape");
}

}  // namespace lbx
