// Block-tiled streaming kernels for large systems of equal-level subsystems
// (the eight-qutrit ring is the design case): lindblad_apply, the stage-solve
// sweeps and the gradient integrands of a single streamed system whose
// subsystems all have NL levels, in one of the LBX_TILE_SHAPES (tile_kernel,
// tile_grad_kernel), and the multi-pass variant (pass_kernel, LB_OPT_TILE 2).
#include <hip/hip_runtime.h>

#include "lbx_host.hpp"

namespace lbx {

constexpr int TILE_BLOCK = 512;  // threads of the multi-pass kernels

namespace {

// sqrt(k) for 0 <= k <= NL as a select chain (k varies per lane).
template <int NL>
__device__ __forceinline__ double sqrt_small(int k) {
  double r = 0.0;
  if (k == 1) r = 1.0;
  if (NL >= 2 && k == 2) r = 1.4142135623730951;
  if (NL >= 3 && k == 3) r = 1.7320508075688772;
  if (NL >= 4 && k == 4) r = 2.0;
  return r;
}

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Value of lane l (uniform l) of a double / int64.
__device__ __forceinline__ double lane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t lane_i64(int64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Every off-diagonal term is a complex multiple of one neighbour value.  With
// d = a + i b the control of subsystem q, the forward control commutator
// contributes
//   row shift +e (weight sqrt(n+1)):  (b, -a) x_{i+e,j}
//   row shift -e (weight sqrt(n)):    (-b, -a) x_{i-e,j}
//   column shift +e (sqrt(m+1)):      (b, a) x_{i,j+e}
//   column shift -e (sqrt(m)):        (-b, a) x_{i,j-e}
// times the weight, and the adjoint the negatives; the decay jump
// contributes g1 sqrt((n+1)(m+1)) x_{i+e,j+e} (adjoint: g1 sqrt(nm) x_{i-e,j-e}).
// These are the terms of `offdiag` in lbx_device.hpp regrouped by neighbour.
enum { DIR_RP = 0, DIR_RM = 1, DIR_CP = 2, DIR_CM = 3 };

template <int DIR, bool ADJ>
__device__ __forceinline__ double2 ctl_coef(double a, double b, double wgt) {
  const double s = ADJ ? -wgt : wgt;
  if (DIR == DIR_RP) return make_double2(s * b, -s * a);
  if (DIR == DIR_RM) return make_double2(-s * b, -s * a);
  if (DIR == DIR_CP) return make_double2(s * b, s * a);
  return make_double2(-s * b, s * a);
}

__device__ __forceinline__ void cmac(double2 &acc, double2 c, double2 v) {
  acc.x += c.x * v.x - c.y * v.y;
  acc.y += c.x * v.y + c.y * v.x;
}

}  // namespace

// MODE 0: y = M x (or M^+ x).  MODE 1: out = q + delta.  MODE 2: out = q + 2 delta,
// delta = w (h D q + h O zin) as in sweep_kernel.
//
// A workgroup owns one TR x TC block of a state, TR = NL^KR rows and
// TC = NL^KC columns: the KR (KC) least significant digits of the row
// (column) index vary and the others are fixed.  The block is staged in LDS,
// so every neighbour along an internal digit (row or column ladder shift, or
// decay jump of a subsystem internal in both) is an LDS read.  Along the
// external digits every neighbour of the block is the block shifted by a
// constant offset, with a coefficient that depends only on the fixed digits.
// Each wavefront tabulates those directions, one per lane (existence,
// coefficient, shift), and walks the existing ones from the ballot mask with
// readlane, G directions at a time: G coalesced loads per entry of a thread
// are in flight together, the neighbour values need no per-entry weights,
// and no direction that does not exist for the block is loaded.  The
// block's own loads are all issued before its LDS stores.  Jumps of a
// subsystem with one internal and one external digit are per-entry global
// loads.  Blocks are remapped so that each XCD (blocks are dealt to the 8
// XCDs round-robin) walks a contiguous band of block rows.
template <int NL, int QC, int KR, int KC, bool ADJ, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tile_kernel(
    const SysDev *__restrict__ sysv, int sys, int64_t nblocks, const double *__restrict__ Etab,
    const double *__restrict__ alpha, const double *__restrict__ carrier, double t,
    const double2 *__restrict__ ctab, int jstep, const double2 *__restrict__ zin,
    const double2 *__restrict__ qin, double2 *__restrict__ out, double2 *__restrict__ zout) {
  extern __shared__ double2 tile[];
  constexpr int ER = QC - KR, EC = QC - KC;  // external row / column digits
  constexpr int TR = ipow(NL, KR), TC = ipow(NL, KC);
  constexpr int TT = TR * TC;
  constexpr int EPT = (TT + BLOCK - 1) / BLOCK;
  // External direction slots: two ladder shifts per external digit and one
  // jump per subsystem external in both (at most 40 for 8 subsystems), one
  // per lane; the existing ones are applied G at a time.
  constexpr int ND = 2 * ER + 2 * EC + (ER < EC ? ER : EC);
  static_assert(ND < 64, "one lane per direction slot, and a lane without one");
  constexpr int G = EPT >= 8 ? 1 : EPT >= 4 ? 2 : 4;
  constexpr bool TABLE = EPT > 1 && EPT < 12;
  const SysDev &S = sysv[sys];
  const int N = S.N;
  const int NBR = N / TR, NBC = N / TC;
  const int64_t N2 = S.N2;
  const int tid = threadIdx.x;
  const int64_t per = (nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= nblocks) return;
  const int64_t b = lb / ((int64_t)NBR * NBC);
  const int rem = (int)(lb - b * NBR * NBC);
  const int bi = rem / NBC, bj = rem - (rem / NBC) * NBC;
  const double2 *X = zin + b * N2;
  const int64_t base = (int64_t)bi * TR * N + (int64_t)bj * TC;
  // flat offset (within the state) of this thread's k-th entry
  auto off_of = [&](int k) -> int64_t {
    const int f = tid + k * BLOCK;
    const int ff = f < TT ? f : 0;
    const int a = ff / TC, c = ff - (ff / TC) * TC;
    return base + (int64_t)a * N + c;
  };
  // fixed (external) digits of the row and column index
  int ne[ER > 0 ? ER : 1], me[EC > 0 ? EC : 1];
  {
    int ri = bi;
#pragma unroll
    for (int q = ER - 1; q >= 0; --q) {
      ne[q] = ri % NL;
      ri /= NL;
    }
    int rj = bj;
#pragma unroll
    for (int q = EC - 1; q >= 0; --q) {
      me[q] = rj % NL;
      rj /= NL;
    }
  }
  // Every wavefront forms the controls, lane q holding d_q: the apply (MODE
  // 0) evaluates them before the block's loads, so that no loaded value is
  // live across the evaluation; the sweeps read them from the control table.
  const int lane = tid & 63;
  double2 dv = make_double2(0.0, 0.0);
  if (MODE == 0 && lane < QC) dv = control_value(S, alpha, carrier + S.carrier_off, lane, t);
  int64_t offs[EPT];
  double2 tv[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {  // (past the block's end: entry 0, unused)
    offs[k] = off_of(k);
    tv[k] = X[offs[k]];
  }
  if (MODE != 0 && lane < QC) dv = ctab[S.ctab_off + (int64_t)jstep * QC + lane];
  double da[QC], db[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    da[q] = lane_d(dv.x, q);
    db[q] = lane_d(dv.y, q);
  }
  // While the block loads, every wavefront builds its table of external
  // directions (blocks of 2 to 11 entries per thread): lane d takes slot
  // d (row digit d / 2, column digit (d - 2 ER) / 2, then jumps) and decides
  // whether its neighbour exists for this block, with its coefficient and
  // shift.
  bool ex = false;
  double2 cf = make_double2(0.0, 0.0);
  int64_t sh = 0;
  if constexpr (TABLE) {
    if (lane < ND) {
      const int d = lane;
      const int kind = d < 2 * ER ? 0 : d < 2 * ER + 2 * EC ? 1 : 2;
      const int q = kind == 0 ? d >> 1 : kind == 1 ? (d - 2 * ER) >> 1 : d - 2 * ER - 2 * EC;
      const bool plus = kind == 2 || !(d & 1);
      int n = 0, m = 0;
      int64_t st = 0;
      double g1 = 0.0, a = 0.0, bq = 0.0;
#pragma unroll
      for (int qq = 0; qq < QC; ++qq)
        if (q == qq) {
          st = S.stride[qq];
          g1 = S.g1[qq];
          a = da[qq];
          bq = db[qq];
        }
#pragma unroll
      for (int qq = 0; qq < ER; ++qq)
        if (q == qq) n = ne[qq];
#pragma unroll
      for (int qq = 0; qq < EC; ++qq)
        if (q == qq) m = me[qq];
      if (kind == 0) {
        ex = plus ? n + 1 < NL : n > 0;
        cf = plus ? ctl_coef<DIR_RP, ADJ>(a, bq, sqrt_small<NL>(n + 1))
                  : ctl_coef<DIR_RM, ADJ>(a, bq, sqrt_small<NL>(n));
        sh = plus ? st * N : -st * N;
      } else if (kind == 1) {
        ex = plus ? m + 1 < NL : m > 0;
        cf = plus ? ctl_coef<DIR_CP, ADJ>(a, bq, sqrt_small<NL>(m + 1))
                  : ctl_coef<DIR_CM, ADJ>(a, bq, sqrt_small<NL>(m));
        sh = plus ? st : -st;
      } else {
        ex = !ADJ ? (n + 1 < NL && m + 1 < NL) : (n > 0 && m > 0);
        cf = make_double2(!ADJ ? g1 * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1)
                               : g1 * sqrt_small<NL>(n) * sqrt_small<NL>(m),
                          0.0);
        sh = !ADJ ? st * N + st : -(st * N + st);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int f = tid + k * BLOCK;
    if (f < TT) tile[f] = tv[k];
  }
  const double h = S.h;
  const double *Es = Etab + S.tab_off;
  // External directions first (they do not read the LDS block), G at a time:
  // the existing slots are taken in order from the ballot mask, a missing
  // G-th one is the last lane (no slot: weight zero, shift zero); one
  // coalesced load per entry of the thread and direction, G x EPT in flight.
  double2 acc[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) acc[k] = make_double2(0.0, 0.0);
  if constexpr (TABLE) {
    uint64_t emask = __ballot(ex);
    while (emask) {
      int dl[G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        dl[g] = emask ? (int)__builtin_ctzll(emask) : 63;
        emask &= emask - 1;
      }
      double2 cg[G], v[G][EPT];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int64_t s = lane_i64(sh, dl[g]);
#pragma unroll
        for (int k = 0; k < EPT; ++k) v[g][k] = X[offs[k] + s];
      }
#pragma unroll
      for (int g = 0; g < G; ++g) cg[g] = make_double2(lane_d(cf.x, dl[g]), lane_d(cf.y, dl[g]));
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < EPT; ++k) cmac(acc[k], cg[g], v[g][k]);
    }
  } else {
    // One entry per thread, or the largest blocks: the directions one at a
    // time under uniform branches (measured faster there than the table).
    auto direction = [&](double2 c, int64_t shift) {
#pragma unroll
      for (int k = 0; k < EPT; ++k) cmac(acc[k], c, X[offs[k] + shift]);
    };
#pragma unroll
    for (int q = 0; q < ER; ++q) {
      const int n = ne[q];
      const int64_t sN = (int64_t)S.stride[q] * N;
      if (n + 1 < NL) direction(ctl_coef<DIR_RP, ADJ>(da[q], db[q], sqrt_small<NL>(n + 1)), sN);
      if (n > 0) direction(ctl_coef<DIR_RM, ADJ>(da[q], db[q], sqrt_small<NL>(n)), -sN);
    }
#pragma unroll
    for (int q = 0; q < EC; ++q) {
      const int m = me[q];
      const int64_t s1 = S.stride[q];
      if (m + 1 < NL) direction(ctl_coef<DIR_CP, ADJ>(da[q], db[q], sqrt_small<NL>(m + 1)), s1);
      if (m > 0) direction(ctl_coef<DIR_CM, ADJ>(da[q], db[q], sqrt_small<NL>(m)), -s1);
    }
#pragma unroll
    for (int q = 0; q < (ER < EC ? ER : EC); ++q) {
      const int n = ne[q], m = me[q];
      const bool jr = !ADJ ? (n + 1 < NL && m + 1 < NL) : (n > 0 && m > 0);
      if (jr) {
        const double cj = !ADJ ? S.g1[q] * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1)
                               : S.g1[q] * sqrt_small<NL>(n) * sqrt_small<NL>(m);
        const int64_t sj = (int64_t)S.stride[q] * N + S.stride[q];
        direction(make_double2(cj, 0.0), !ADJ ? sj : -sj);
      }
    }
  }
  __syncthreads();
  // Internal terms (LDS), the diagonal part and the output, entry by entry.
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int f = tid + k * BLOCK;
    if (f >= TT) continue;
    const int a = f / TC, c = f - (f / TC) * TC;
    int nd[QC], md[QC];
    {
      int ra = a;
#pragma unroll
      for (int q = QC - 1; q >= ER; --q) {
        nd[q] = ra % NL;
        ra /= NL;
      }
#pragma unroll
      for (int q = 0; q < ER; ++q) nd[q] = ne[q];
      int rc = c;
#pragma unroll
      for (int q = QC - 1; q >= EC; --q) {
        md[q] = rc % NL;
        rc /= NL;
      }
#pragma unroll
      for (int q = 0; q < EC; ++q) md[q] = me[q];
    }
    double gam = 0.0;
    double2 ac = acc[k];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int n = nd[q], m = md[q];
      const double dnm = (double)(n - m);
      gam += 0.5 * (S.g1[q] * (double)(n + m) + S.g2[q] * dnm * dnm);
      const int st = S.stride[q];
      // Internal neighbours are LDS reads; a missing one reads the entry
      // itself with a zero weight (no divergent branches).
      const bool rp = n + 1 < NL, rm = n > 0, cp = m + 1 < NL, cm = m > 0;
      if (q >= ER) {  // internal row digit: a row shift of st is st*TC entries in the block
        cmac(ac, ctl_coef<DIR_RP, ADJ>(da[q], db[q], rp ? sqrt_small<NL>(n + 1) : 0.0),
             tile[f + (rp ? st * TC : 0)]);
        cmac(ac, ctl_coef<DIR_RM, ADJ>(da[q], db[q], sqrt_small<NL>(n)), tile[f - (rm ? st * TC : 0)]);
      }
      if (q >= EC) {
        cmac(ac, ctl_coef<DIR_CP, ADJ>(da[q], db[q], cp ? sqrt_small<NL>(m + 1) : 0.0),
             tile[f + (cp ? st : 0)]);
        cmac(ac, ctl_coef<DIR_CM, ADJ>(da[q], db[q], sqrt_small<NL>(m)), tile[f - (cm ? st : 0)]);
      }
      const bool jr = !ADJ ? (rp && cp) : (rm && cm);
      const double cj = !jr ? 0.0
                            : !ADJ ? S.g1[q] * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1)
                                   : S.g1[q] * sqrt_small<NL>(n) * sqrt_small<NL>(m);
      if (q >= ER && q >= EC) {
        const double2 v = tile[f + (!jr ? 0 : !ADJ ? st * TC + st : -(st * TC + st))];
        ac.x += cj * v.x;
        ac.y += cj * v.y;
      } else if (q >= ER || q >= EC) {  // one digit internal: a per-entry global load
        const int64_t sj = (int64_t)st * N + st;
        const double2 v = X[offs[k] + (!jr ? 0 : !ADJ ? sj : -sj)];
        ac.x += cj * v.x;
        ac.y += cj * v.y;
      }
    }
    const int i = bi * TR + a, j = bj * TC + c;
    const double dE = Es[i] - Es[j];
    const double2 D = diag_coef(gam, dE, ADJ);
    const int64_t e = b * N2 + offs[k];
    if (MODE == 0) {
      out[e] = cadd(ac, cmul(D, tile[f]));
    } else {
      const double2 qv = qin[e];
      const double2 w = stage_weight(h, gam, dE, ADJ);
      const double2 hdq = cscale(h, cmul(D, qv));
      const double2 dn = cmul(w, make_double2(hdq.x + h * ac.x, hdq.y + h * ac.y));
      out[e] = MODE == 2 ? make_double2(qv.x + 2.0 * dn.x, qv.y + 2.0 * dn.y) : cadd(qv, dn);
      if (MODE == 2 && zout) zout[e] = cadd(qv, dn);  // the converged stage vector
    }
  }
}

// Gradient integrands of one step (App. B eq. reducedgradient) with the same
// blocking as tile_kernel: zh (the adjoint stage vector) is staged in LDS,
// the forward stage vector z = (q0 + q1)/2 is read per entry, and for every
// subsystem q the block sums
//   gp_q = sum Re<X_q zh, z>-type terms  and  gq_q likewise
// as in grad_term (lbx_device.hpp), regrouped by neighbour: with U and V
// built from the ladder neighbours of zh, gp += cross(U + V, z) and
// gq -= dot(U - V, z), cross(a, z) = a.x z.y - a.y z.x.  Neighbours along
// external digits are applied one direction at a time.  One row of 2 QMAX
// partial sums per block.
__device__ __forceinline__ double cross2(double2 a, double2 z) { return a.x * z.y - a.y * z.x; }
__device__ __forceinline__ double dot2(double2 a, double2 z) { return a.x * z.x + a.y * z.y; }

template <int NL, int QC, int KR, int KC, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tile_grad_kernel(
    const SysDev *__restrict__ sysv, int sys, int64_t nblocks, const double2 *__restrict__ zh,
    const double2 *__restrict__ q0, const double2 *__restrict__ q1, double *__restrict__ gpart) {
  extern __shared__ double2 tile[];
  __shared__ double red[BLOCK / 64][2 * QC];
  constexpr int ER = QC - KR, EC = QC - KC;
  constexpr int TR = ipow(NL, KR), TC = ipow(NL, KC);
  constexpr int TT = TR * TC;
  constexpr int EPT = (TT + BLOCK - 1) / BLOCK;
  const SysDev &S = sysv[sys];
  const int N = S.N;
  const int NBR = N / TR, NBC = N / TC;
  const int64_t N2 = S.N2;
  const int tid = threadIdx.x;
  const int64_t per = (nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= nblocks) return;
  const int64_t b = lb / ((int64_t)NBR * NBC);
  const int rem = (int)(lb - b * NBR * NBC);
  const int bi = rem / NBC, bj = rem - (rem / NBC) * NBC;
  const double2 *Z = zh + b * N2;
  const int64_t base = (int64_t)bi * TR * N + (int64_t)bj * TC;
  auto off_of = [&](int k) -> int64_t {
    const int f = tid + k * BLOCK;
    const int ff = f < TT ? f : 0;
    const int a = ff / TC, c = ff - (ff / TC) * TC;
    return base + (int64_t)a * N + c;
  };
  double2 z[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int f = tid + k * BLOCK;
    const int64_t e = off_of(k);  // (past the block's end: entry 0, unused)
    const double2 v = Z[e];
    const double2 a = q0[b * N2 + e], c = q1[b * N2 + e];
    if (f < TT) tile[f] = v;
    z[k] = f < TT ? make_double2(0.5 * (a.x + c.x), 0.5 * (a.y + c.y)) : make_double2(0.0, 0.0);
  }
  int ne[ER > 0 ? ER : 1], me[EC > 0 ? EC : 1];
  {
    int ri = bi;
#pragma unroll
    for (int q = ER - 1; q >= 0; --q) {
      ne[q] = ri % NL;
      ri /= NL;
    }
    int rj = bj;
#pragma unroll
    for (int q = EC - 1; q >= 0; --q) {
      me[q] = rj % NL;
      rj /= NL;
    }
  }
  __syncthreads();
  double gp[QC], gq[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) gp[q] = gq[q] = 0.0;
  // external directions; sp, sq: signs of the cross and dot terms
  auto direction = [&](int q, double w, double sp, double sg, int64_t shift) {
    double2 v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) v[k] = Z[off_of(k) + shift];
    double cp = 0.0, dp = 0.0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      cp += cross2(v[k], z[k]);
      dp += dot2(v[k], z[k]);
    }
    gp[q] += sp * w * cp;
    gq[q] += sg * w * dp;
  };
#pragma unroll
  for (int q = 0; q < ER; ++q) {
    const int n = ne[q];
    const int64_t sN = (int64_t)S.stride[q] * N;
    if (n + 1 < NL) direction(q, sqrt_small<NL>(n + 1), 1.0, -1.0, sN);   // U += sqrt(n+1) x_{i+e}
    if (n > 0) direction(q, sqrt_small<NL>(n), 1.0, 1.0, -sN);            // V += sqrt(n) x_{i-e}
  }
#pragma unroll
  for (int q = 0; q < EC; ++q) {
    const int m = me[q];
    const int64_t s1 = S.stride[q];
    if (m + 1 < NL) direction(q, sqrt_small<NL>(m + 1), -1.0, -1.0, s1);  // V -= sqrt(m+1) x_{j+e}
    if (m > 0) direction(q, sqrt_small<NL>(m), -1.0, 1.0, -s1);           // U -= sqrt(m) x_{j-e}
  }
  // internal neighbours from LDS
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int f = tid + k * BLOCK;
    if (f >= TT) continue;
    const int a = f / TC, c = f - (f / TC) * TC;
    int ra = a, rc = c;
#pragma unroll
    for (int q = QC - 1; q >= 0; --q) {
      const int st = S.stride[q];
      if (q >= ER) {
        const int n = ra % NL;
        ra /= NL;
        const bool rp = n + 1 < NL, rm = n > 0;
        const double2 vp = tile[f + (rp ? st * TC : 0)], vm = tile[f - (rm ? st * TC : 0)];
        const double wp = rp ? sqrt_small<NL>(n + 1) : 0.0, wm = sqrt_small<NL>(n);
        gp[q] += wp * cross2(vp, z[k]) + wm * cross2(vm, z[k]);
        gq[q] += -wp * dot2(vp, z[k]) + wm * dot2(vm, z[k]);
      }
      if (q >= EC) {
        const int m = rc % NL;
        rc /= NL;
        const bool cp = m + 1 < NL, cm = m > 0;
        const double2 vp = tile[f + (cp ? st : 0)], vm = tile[f - (cm ? st : 0)];
        const double wp = cp ? sqrt_small<NL>(m + 1) : 0.0, wm = sqrt_small<NL>(m);
        gp[q] += -wp * cross2(vp, z[k]) - wm * cross2(vm, z[k]);
        gq[q] += -wp * dot2(vp, z[k]) + wm * dot2(vm, z[k]);
      }
    }
  }
  // block sums in a fixed order
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    const double a = wave_sum<64>(gp[q]), c = wave_sum<64>(gq[q]);
    if (lane == 0) {
      red[wv][2 * q] = a;
      red[wv][2 * q + 1] = c;
    }
  }
  __syncthreads();
  if (tid < 2 * QC) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) v += red[w][tid];
    gpart[lb * 2 * QMAX + tid] = v;
  }
}

// Multi-pass application for large systems of equal-level subsystems.  The
// subsystems are split into groups; pass g applies the terms of group g
// (row and column ladder shifts and decay jumps, all of which move only
// digits of the group's subsystems) to every entry, so that a block holding
// every row digit of the group in its rows (mask RM) and every column digit
// in its columns (mask CM) finds all neighbours in LDS and reads nothing
// outside itself.  Both masks may hold further, passive digits: the lowest
// column digits are always in CM, so that a block row is a contiguous run
// of at least 16 entries.  The first pass writes its terms to `out`, later
// passes add theirs to what `out` holds (each entry is read and written by
// one thread), and the last adds the diagonal part (MODE 0) or takes the
// stage update (MODE 1, 2); out must therefore not overlap zin or qin.
// Bit q of a mask stands for subsystem q (q = 0 most significant).
constexpr int popc(unsigned m) { return m ? (int)(m & 1u) + popc(m >> 1) : 0; }

template <int NL, int QC, unsigned IM, unsigned RM, unsigned CM, int STAGE, bool ADJ, int MODE>
__global__ __launch_bounds__(TILE_BLOCK) void pass_kernel(
    const SysDev *__restrict__ sysv, int sys, int64_t nblocks, const double *__restrict__ Etab,
    const double *__restrict__ alpha, const double *__restrict__ carrier, double t,
    const double2 *__restrict__ ctab, int jstep, const double2 *__restrict__ zin,
    const double2 *__restrict__ qin, double2 *__restrict__ out, double2 *__restrict__ zout) {
  extern __shared__ double2 tile[];
  __shared__ double2 dqs[QC];
  constexpr int NR = popc(RM), NC = popc(CM);
  constexpr int TRn = ipow(NL, NR), TCn = ipow(NL, NC), TT = TRn * TCn;
  constexpr int FC = ipow(NL, QC - NC), FR = ipow(NL, QC - NR);
  constexpr int EPT = (TT + TILE_BLOCK - 1) / TILE_BLOCK;
  const SysDev &S = sysv[sys];
  const int N = S.N;
  const int64_t N2 = S.N2;
  const int tid = threadIdx.x;
  const int64_t per = (nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= nblocks) return;
  if (tid < QC)
    dqs[tid] = ctab ? ctab[S.ctab_off + (int64_t)jstep * QC + tid]
                    : control_value(S, alpha, carrier + S.carrier_off, tid, t);
  const int64_t b = lb / ((int64_t)FR * FC);
  const int rem = (int)(lb - b * FR * FC);
  // fixed digits: the row digits outside RM from u, the column digits outside CM from v
  int nf[QC], mf[QC];
  int ibase = 0, jbase = 0;
  {
    int u = rem / FC, v = rem - (rem / FC) * FC;
#pragma unroll
    for (int q = QC - 1; q >= 0; --q) {
        const int sq = ipow(NL, QC - 1 - q);
      if (!((RM >> q) & 1u)) {
        nf[q] = u % NL;
        u /= NL;
        ibase += nf[q] * sq;
      } else {
        nf[q] = 0;
      }
      if (!((CM >> q) & 1u)) {
        mf[q] = v % NL;
        v /= NL;
        jbase += mf[q] * sq;
      } else {
        mf[q] = 0;
      }
    }
  }
  const double2 *X = zin + b * N2;
  // row / column offset of block row a / block column c, and all digits
  auto rowoff = [&](int a) {
    int r = 0;
#pragma unroll
    for (int q = QC - 1; q >= 0; --q)
      if ((RM >> q) & 1u) {
        r += (a % NL) * ipow(NL, QC - 1 - q);
        a /= NL;
      }
    return r;
  };
  auto coloff = [&](int c) {
    int r = 0;
#pragma unroll
    for (int q = QC - 1; q >= 0; --q)
      if ((CM >> q) & 1u) {
        r += (c % NL) * ipow(NL, QC - 1 - q);
        c /= NL;
      }
    return r;
  };
  auto off_of = [&](int k) -> int64_t {
    const int f = tid + k * TILE_BLOCK;
    const int ff = f < TT ? f : 0;
    const int a = ff / TCn, c = ff - (ff / TCn) * TCn;
    return (int64_t)(ibase + rowoff(a)) * N + jbase + coloff(c);
  };
  {
    double2 tv[EPT];  // all loads in flight before the first LDS store
#pragma unroll
    for (int k = 0; k < EPT; ++k) tv[k] = X[off_of(k)];  // (past the end: entry 0, unused)
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int f = tid + k * TILE_BLOCK;
      if (f < TT) tile[f] = tv[k];
    }
  }
  const double h = S.h;
  const double *Es = Etab + S.tab_off;
  __syncthreads();
  double da[QC], db[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    da[q] = uniform(dqs[q].x);
    db[q] = uniform(dqs[q].y);
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int f = tid + k * TILE_BLOCK;
    if (f >= TT) continue;
    const int a = f / TCn, c = f - (f / TCn) * TCn;
    int nd[QC], md[QC];
    {
      int ra = a, rc = c;
#pragma unroll
      for (int q = QC - 1; q >= 0; --q) {
        if ((RM >> q) & 1u) {
          nd[q] = ra % NL;
          ra /= NL;
        } else {
          nd[q] = nf[q];
        }
        if ((CM >> q) & 1u) {
          md[q] = rc % NL;
          rc /= NL;
        } else {
          md[q] = mf[q];
        }
      }
    }
    double2 ac = make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      if (!((IM >> q) & 1u)) continue;
      const int n = nd[q], m = md[q];
      // strides of digit q inside the block's row and column index
      const int sr = ipow(NL, popc(RM & (~0u << (q + 1)))) * TCn;
      const int sc = ipow(NL, popc(CM & (~0u << (q + 1))));
      const bool rp = n + 1 < NL, rm = n > 0, cp = m + 1 < NL, cm = m > 0;
      cmac(ac, ctl_coef<DIR_RP, ADJ>(da[q], db[q], rp ? sqrt_small<NL>(n + 1) : 0.0), tile[f + (rp ? sr : 0)]);
      cmac(ac, ctl_coef<DIR_RM, ADJ>(da[q], db[q], sqrt_small<NL>(n)), tile[f - (rm ? sr : 0)]);
      cmac(ac, ctl_coef<DIR_CP, ADJ>(da[q], db[q], cp ? sqrt_small<NL>(m + 1) : 0.0), tile[f + (cp ? sc : 0)]);
      cmac(ac, ctl_coef<DIR_CM, ADJ>(da[q], db[q], sqrt_small<NL>(m)), tile[f - (cm ? sc : 0)]);
      const bool jr = !ADJ ? (rp && cp) : (rm && cm);
      const double cj = !jr ? 0.0
                            : !ADJ ? S.g1[q] * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1)
                                   : S.g1[q] * sqrt_small<NL>(n) * sqrt_small<NL>(m);
      const double2 vj = tile[f + (!jr ? 0 : !ADJ ? sr + sc : -(sr + sc))];
      ac.x += cj * vj.x;
      ac.y += cj * vj.y;
    }
    const int i = ibase + rowoff(a), j = jbase + coloff(c);
    const int64_t e = b * N2 + (int64_t)i * N + j;
    if (STAGE == 0) {
      out[e] = ac;
      continue;
    }
    ac = cadd(ac, out[e]);
    if (STAGE == 1) {
      out[e] = ac;
      continue;
    }
    double gam = 0.0;
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const double dnm = (double)(nd[q] - md[q]);
      gam += 0.5 * (S.g1[q] * (double)(nd[q] + md[q]) + S.g2[q] * dnm * dnm);
    }
    const double dE = Es[i] - Es[j];
    const double2 D = diag_coef(gam, dE, ADJ);
    if (MODE == 0) {
      out[e] = cadd(ac, cmul(D, tile[f]));
    } else {
      const double2 qv = qin[e];
      const double2 w = stage_weight(h, gam, dE, ADJ);
      const double2 hdq = cscale(h, cmul(D, qv));
      const double2 dn = cmul(w, make_double2(hdq.x + h * ac.x, hdq.y + h * ac.y));
      out[e] = MODE == 2 ? make_double2(qv.x + 2.0 * dn.x, qv.y + 2.0 * dn.y) : cadd(qv, dn);
      if (MODE == 2 && zout) zout[e] = cadd(qv, dn);  // the converged stage vector
    }
  }
}

template <int NL, int QC, unsigned IM, unsigned RM, unsigned CM, int STAGE, bool ADJ, int MODE>
static int pass_launch(const lb_plan *p, int sys, int B, const double *alpha, double t,
                       const double2 *ctab, int j, const double2 *zin, const double2 *qin,
                       double2 *out, double2 *zout, hipStream_t st) {
  constexpr int NR = popc(RM), NC = popc(CM);
  static_assert(ipow(NL, NR + NC) <= 6561, "block does not fit in LDS");
  const size_t shmem = (size_t)ipow(NL, NR + NC) * sizeof(double2);
  auto kern = pass_kernel<NL, QC, IM, RM, CM, STAGE, ADJ, MODE>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const int64_t nblocks = (int64_t)B * ipow(NL, QC - NR) * ipow(NL, QC - NC);
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(TILE_BLOCK), shmem, st, p->d_sys, sys, nblocks,
                     p->d_E, alpha, p->d_carrier, t, ctab, j, zin, qin, out, zout);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

// One pass of a plan: STAGE 0 first, 1 middle, 2 last (which takes MODE).
template <int NL, int QC, unsigned IM, unsigned RM, unsigned CM, int STAGE>
static int pass_run(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha,
                    double t, const double2 *ctab, int j, const double2 *zin, const double2 *qin,
                    double2 *out, double2 *zout, hipStream_t st) {
  if constexpr (STAGE < 2) {
    return adj ? pass_launch<NL, QC, IM, RM, CM, STAGE, true, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st)
               : pass_launch<NL, QC, IM, RM, CM, STAGE, false, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
  }
  if (adj) {
    if (mode == 0) return pass_launch<NL, QC, IM, RM, CM, 2, true, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
    if (mode == 1) return pass_launch<NL, QC, IM, RM, CM, 2, true, 1>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
    return pass_launch<NL, QC, IM, RM, CM, 2, true, 2>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
  }
  if (mode == 0) return pass_launch<NL, QC, IM, RM, CM, 2, false, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
  if (mode == 1) return pass_launch<NL, QC, IM, RM, CM, 2, false, 1>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
  return pass_launch<NL, QC, IM, RM, CM, 2, false, 2>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
}

// Pass plans (NL, Q, then per pass: subsystems applied, row mask, column
// mask).  Every subsystem is applied by exactly one pass.
#define LBX_PASS_PLANS(P3)                                                    \
  P3(3, 8, 0xF0u, 0xF0u, 0xF0u, 0x03u, 0x03u, 0xF3u, 0x0Cu, 0x0Cu, 0xFCu)     \
  P3(3, 7, 0x78u, 0x78u, 0x78u, 0x03u, 0x03u, 0x7Bu, 0x04u, 0x1Cu, 0x7Cu)     \
  P3(2, 12, 0xFC0u, 0xFC0u, 0xFC0u, 0x007u, 0x007u, 0xFC7u, 0x038u, 0x038u, 0xFF8u) \
  P3(2, 11, 0x7E0u, 0x7E0u, 0x7E0u, 0x007u, 0x007u, 0x7E7u, 0x018u, 0x078u, 0x7F8u) \
  P3(4, 6, 0x38u, 0x38u, 0x38u, 0x03u, 0x03u, 0x33u, 0x04u, 0x0Cu, 0x3Cu)

int split_kl(const lb_plan *p, int sys) {
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0];
  for (int q = 1; q < S.Q; ++q)
    if (S.nlev[q] != nl) return 0;
#define P3(A, B, I0, R0, C0, I1, R1, C1, I2, R2, C2) \
  if (nl == A && S.Q == B) return 3;
  LBX_PASS_PLANS(P3)
#undef P3
  return 0;
}

int launch_split(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha, double t,
                 const double2 *ctab, int j, const double2 *zin, const double2 *qin, double2 *out,
                 double2 *zout, hipStream_t st) {
  if (B == 0) return LB_OK;
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0];
  if (!split_kl(p, sys)) return fail(LB_EUNSUPPORTED, "system not eligible for the multi-pass kernels");
#define P3(A, Bq, I0, R0, C0, I1, R1, C1, I2, R2, C2)                                                    \
  if (nl == A && S.Q == Bq) {                                                                           \
    int rc = pass_run<A, Bq, I0, R0, C0, 0>(p, sys, B, mode, adj, alpha, t, ctab, j, zin, qin, out, zout, st); \
    if (!rc) rc = pass_run<A, Bq, I1, R1, C1, 1>(p, sys, B, mode, adj, alpha, t, ctab, j, zin, qin, out, zout, st); \
    if (!rc) rc = pass_run<A, Bq, I2, R2, C2, 2>(p, sys, B, mode, adj, alpha, t, ctab, j, zin, qin, out, zout, st); \
    return rc;                                                                                          \
  }
  LBX_PASS_PLANS(P3)
#undef P3
  return fail(LB_EUNSUPPORTED, "system not eligible for the multi-pass kernels");
}

// Block shapes: KR row digits and KC column digits inside a block.  The
// default is the shape listed first in LBX_TILE_SHAPES for the system (the
// largest square block, at most 6561 entries); the plan's LB_OPT_TILE_KI
// selects another instantiated shape (encoded 10*KR + KC).

template <int NL, int QC, int KR, int KC, int BLOCK, bool ADJ, int MODE>
static int tile_launch(const lb_plan *p, int sys, int B, const double *alpha, double t,
                       const double2 *ctab, int j, const double2 *zin, const double2 *qin,
                       double2 *out, double2 *zout, hipStream_t st) {
  constexpr int TR = ipow(NL, KR), TC = ipow(NL, KC);
  const int N = p->sys[sys].N;
  const size_t shmem = (size_t)TR * TC * sizeof(double2);
  auto kern = tile_kernel<NL, QC, KR, KC, ADJ, MODE, BLOCK>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const int64_t nblocks = (int64_t)B * (N / TR) * (N / TC);
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(BLOCK), shmem, st, p->d_sys, sys, nblocks,
                     p->d_E, alpha, p->d_carrier, t, ctab, j, zin, qin, out, zout);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

template <int NL, int QC, int KR, int KC, int BLOCK>
static int tile_modes(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha,
                      double t, const double2 *ctab, int j, const double2 *zin, const double2 *qin,
                      double2 *out, double2 *zout, hipStream_t st) {
  if (adj) {
    if (mode == 0) return tile_launch<NL, QC, KR, KC, BLOCK, true, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
    if (mode == 1) return tile_launch<NL, QC, KR, KC, BLOCK, true, 1>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
    return tile_launch<NL, QC, KR, KC, BLOCK, true, 2>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
  }
  if (mode == 0) return tile_launch<NL, QC, KR, KC, BLOCK, false, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
  if (mode == 1) return tile_launch<NL, QC, KR, KC, BLOCK, false, 1>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
  return tile_launch<NL, QC, KR, KC, BLOCK, false, 2>(p, sys, B, alpha, t, ctab, j, zin, qin, out, zout, st);
}

// Instantiated shapes (NL, Q, KR, KC, threads per block); the first listed
// for a (NL, Q) is the default.  Blocks of up to 2187 entries run 256
// threads, so that several fit on one compute unit.
#define LBX_TILE_SHAPES(X)                                                                    \
  X(3, 8, 4, 4, 512) X(3, 8, 4, 3, 256) X(3, 8, 3, 4, 256) X(3, 8, 4, 2, 256)                  \
  X(3, 8, 3, 3, 256) X(3, 8, 3, 2, 256) X(3, 8, 2, 3, 256)                                     \
  X(3, 7, 4, 4, 512) X(3, 7, 4, 3, 256) X(3, 7, 3, 3, 256) X(3, 6, 4, 4, 512)                  \
  X(3, 6, 4, 3, 256) X(3, 5, 3, 3, 256) X(3, 5, 3, 2, 256) X(3, 5, 2, 3, 256)                  \
  X(2, 9, 6, 6, 512) X(2, 10, 6, 6, 512) X(2, 11, 6, 6, 512) X(2, 12, 6, 6, 512)               \
  X(4, 5, 3, 3, 512) X(4, 6, 3, 3, 512)

int tile_ki(const lb_plan *p, int sys) {
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0];
  for (int q = 1; q < S.Q; ++q)
    if (S.nlev[q] != nl) return 0;
  int first = 0;
#define X(A, B, R, C, T)                                           \
  if (nl == A && S.Q == B) {                                       \
    if (!first) first = 10 * R + C;                                \
    if (p->tile_ki == 10 * R + C) return 10 * R + C;               \
  }
  LBX_TILE_SHAPES(X)
#undef X
  return first;
}

template <int NL, int QC, int KR, int KC, int BLOCK>
static int tile_grad_launch(const lb_plan *p, int sys, int B, const double2 *zh, const double2 *q0,
                            const double2 *q1, double *gpart, int64_t *rows, hipStream_t st) {
  constexpr int TR = ipow(NL, KR), TC = ipow(NL, KC);
  const int N = p->sys[sys].N;
  const size_t shmem = (size_t)TR * TC * sizeof(double2);
  auto kern = tile_grad_kernel<NL, QC, KR, KC, BLOCK>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const int64_t nblocks = (int64_t)B * (N / TR) * (N / TC);
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(BLOCK), shmem, st, p->d_sys, sys, nblocks, zh, q0,
                     q1, gpart);
  LBX_HIP(hipGetLastError());
  *rows = nblocks;
  return LB_OK;
}

// Gradient integrands of one step for a system on the block-tiled path, in
// the block shape of its sweeps (the single-pass shape even when the sweeps
// use the multi-pass kernels).  *rows receives the number of partial rows.
int launch_tile_grad(const lb_plan *p, int sys, int B, const double2 *zh, const double2 *q0,
                     const double2 *q1, double *gpart, int64_t *rows, hipStream_t st) {
  *rows = 0;
  if (B == 0) return LB_OK;
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0], k = tile_ki(p, sys);
#define X(A, Bq, R, C, T) \
  if (nl == A && S.Q == Bq && k == 10 * R + C) return tile_grad_launch<A, Bq, R, C, T>(p, sys, B, zh, q0, q1, gpart, rows, st);
  LBX_TILE_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "system not eligible for the tiled gradient kernel");
}

int64_t tile_grad_rows(const lb_plan *p, int sys, int B) {
  const SysDev &S = p->sys[sys];
  const int k = tile_ki(p, sys);
  if (!k) return 0;
  int tr = 1, tc = 1;
  for (int i = 0; i < k / 10; ++i) tr *= S.nlev[0];
  for (int i = 0; i < k % 10; ++i) tc *= S.nlev[0];
  return (int64_t)B * (S.N / tr) * (S.N / tc);
}

int tile_nl(const lb_plan *p, int sys) {
  return (tile_ki(p, sys) > 0 || (p->tile == 2 && split_kl(p, sys) > 0)) ? p->sys[sys].nlev[0] : 0;
}

int launch_tile(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha, double t,
                const double2 *ctab, int j, const double2 *zin, const double2 *qin, double2 *out,
                double2 *zout, hipStream_t st) {
  if (B == 0) return LB_OK;
  if (p->tile == 2 && split_kl(p, sys))
    return launch_split(p, sys, B, mode, adj, alpha, t, ctab, j, zin, qin, out, zout, st);
  if (mode != 0 && !ctab) return fail(LB_EINVAL, "stage sweeps need the control table");
  const SysDev &S = p->sys[sys];
  const int nl = tile_nl(p, sys), k = tile_ki(p, sys);
#define X(A, Bq, R, C, T) \
  if (nl == A && S.Q == Bq && k == 10 * R + C) return tile_modes<A, Bq, R, C, T>(p, sys, B, mode, adj, alpha, t, ctab, j, zin, qin, out, zout, st);
  LBX_TILE_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "system not eligible for the tiled kernels");
}

}  // namespace lbx
