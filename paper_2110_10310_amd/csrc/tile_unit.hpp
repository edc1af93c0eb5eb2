// One block-tiled unit of the matrix-free Lindbladian (App. A eq.
// mastereq_vectorized) for a system whose subsystems all have NL levels.
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
// loads.
//
// tile_unit computes, for every entry e of the unit, the off-diagonal sum
// (O x)_e (or (O^+ x)_e) and the diagonal data, and hands them to an output
// functor; the apply kernel, the stage sweeps and the persistent step
// kernels differ only in that functor.
#pragma once

#include "lbx_device.hpp"

namespace lbx {
namespace tile {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

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

template <int NL, int QC, int KR, int KC, int BLOCK>
struct Shape {
  static constexpr int ER = QC - KR, EC = QC - KC;  // external row / column digits
  static constexpr int TR = ipow(NL, KR), TC = ipow(NL, KC);
  static constexpr int TT = TR * TC;
  static constexpr int EPT = (TT + BLOCK - 1) / BLOCK;
  // External direction slots: two ladder shifts per external digit and one
  // jump per subsystem external in both (at most 40 for 8 subsystems), one
  // per lane; the existing ones are applied G at a time.
  static constexpr int ND = 2 * ER + 2 * EC + (ER < EC ? ER : EC);
  static_assert(ND < 64, "one lane per direction slot, and a lane without one");
  static constexpr int G = EPT >= 8 ? 1 : EPT >= 4 ? 2 : 4;
  static constexpr bool TABLE = EPT > 1 && EPT < 12;
  static constexpr size_t lds_bytes() { return (size_t)TT * sizeof(double2); }
};

// Units of one launch are numbered lb = 0 .. B*NBR*NBC - 1 (state-major,
// then block row, then block column).
__host__ __device__ inline int64_t tile_units(int N, int TR, int TC, int B) {
  return (int64_t)B * (N / TR) * (N / TC);
}

// Gradient integrands of one adjoint step (App. B eq. reducedgradient) formed
// alongside a unit: the unit's input x is the adjoint stage vector zh, z =
// (q0 + q1)/2 is the forward stage vector at the unit's own entries, and for
// every subsystem q the thread sums
//   p[q] += w Im-type and q[q] += w Re-type products of x at the q-neighbours
// with z, regrouped by neighbour (the terms of grad_term in lbx_device.hpp).
template <int QC>
struct GradAcc {
  const double2 *q0, *q1;  // forward states q^j and q^{j+1} ([B][N][N])
  double p[QC], q[QC];
};

__device__ __forceinline__ double gcross(double2 a, double2 z) { return a.x * z.y - a.y * z.x; }
__device__ __forceinline__ double gdot(double2 a, double2 z) { return a.x * z.x + a.y * z.y; }

// The data of one entry handed to the output functor.
struct Entry {
  int64_t e;     // flat index of the entry in the batch ([B][N][N])
  int f;         // index of the entry in the unit (LDS slot)
  double2 acc;   // off-diagonal part (O x)_e or (O^+ x)_e
  double2 own;   // x_e
  double gam;    // decay anticommutator + dephasing rate gamma_ij
  double dE;     // E_i - E_j
};

// One unit.  zin: the batch [B][N][N] whose neighbours are read; tile: LDS of
// Shape::TT entries; da, db: real and imaginary controls of every subsystem
// (uniform); Es: energies of this system.  When `sync_first` the workgroup
// waits before its LDS stores (a previous unit in the same workgroup may
// still read the buffer).  out(const Entry &) is called once per entry of
// the unit.  With GRAD the unit also adds this thread's gradient integrands
// with zin as the adjoint stage vector to *ga (the neighbour values the
// stencil loads serve both); the forward stage vector of the unit is then
// staged in LDS after the block (tile must hold 2 TT entries) and the
// external directions are taken one at a time.
template <int NL, int QC, int KR, int KC, bool ADJ, int BLOCK, bool GRAD = false, class Out>
__device__ __forceinline__ void tile_unit(const SysDev &S, int64_t lb, const double2 *__restrict__ zin,
                                          double2 *tile, const double (&da)[QC], const double (&db)[QC],
                                          const double *__restrict__ Es, bool sync_first, Out &&out,
                                          GradAcc<QC> *ga = nullptr) {
  using Sh = Shape<NL, QC, KR, KC, BLOCK>;
  constexpr int ER = Sh::ER, EC = Sh::EC, TR = Sh::TR, TC = Sh::TC, TT = Sh::TT, EPT = Sh::EPT;
  constexpr int ND = Sh::ND, G = GRAD ? 1 : Sh::G;
  constexpr bool TABLE = Sh::TABLE;
  const int N = S.N;
  const int NBR = N / TR, NBC = N / TC;
  const int64_t N2 = S.N2;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
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
  int64_t offs[EPT];
  double2 tv[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {  // (past the block's end: entry 0, unused)
    offs[k] = off_of(k);
    tv[k] = X[offs[k]];
  }
  // forward stage vector at the own entries, staged in LDS with the block
  double2 *const ztile = tile + TT;
  double2 zl[GRAD ? EPT : 1];
  if constexpr (GRAD) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const double2 a = ga->q0[b * N2 + offs[k]], c = ga->q1[b * N2 + offs[k]];
      zl[k] = make_double2(0.5 * (a.x + c.x), 0.5 * (a.y + c.y));
    }
  }
  // forward stage vector of this thread's k-th entry (zero past the block's end)
  auto zf = [&](int k) -> double2 {
    const int f = tid + k * BLOCK;
    return f < TT ? ztile[f] : make_double2(0.0, 0.0);
  };
  // While the block loads, every wavefront builds its table of external
  // directions (blocks of 2 to 11 entries per thread): lane d takes slot
  // d (row digit d / 2, column digit (d - 2 ER) / 2, then jumps) and decides
  // whether its neighbour exists for this block, with its coefficient and
  // shift.
  bool ex = false;
  double2 cf = make_double2(0.0, 0.0);
  int64_t sh = 0;
  double gwp = 0.0, gwq = 0.0;  // GRAD: weights of the direction's integrand terms
  int gqi = 0;                  // GRAD: its subsystem
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
        if constexpr (GRAD) {
          // row shift +e: (w, -w) with w = sqrt(n+1); -e: (w, w) with w = sqrt(n)
          const double w = plus ? sqrt_small<NL>(n + 1) : sqrt_small<NL>(n);
          gwp = w;
          gwq = plus ? -w : w;
          gqi = q;
        }
      } else if (kind == 1) {
        ex = plus ? m + 1 < NL : m > 0;
        cf = plus ? ctl_coef<DIR_CP, ADJ>(a, bq, sqrt_small<NL>(m + 1))
                  : ctl_coef<DIR_CM, ADJ>(a, bq, sqrt_small<NL>(m));
        sh = plus ? st : -st;
        if constexpr (GRAD) {
          // column shift +e: (-w, -w) with w = sqrt(m+1); -e: (-w, w) with w = sqrt(m)
          const double w = plus ? sqrt_small<NL>(m + 1) : sqrt_small<NL>(m);
          gwp = -w;
          gwq = plus ? -w : w;
          gqi = q;
        }
      } else {
        ex = !ADJ ? (n + 1 < NL && m + 1 < NL) : (n > 0 && m > 0);
        cf = make_double2(!ADJ ? g1 * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1)
                               : g1 * sqrt_small<NL>(n) * sqrt_small<NL>(m),
                          0.0);
        sh = !ADJ ? st * N + st : -(st * N + st);
      }
    }
  }
  if (sync_first) __syncthreads();
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int f = tid + k * BLOCK;
    if (f < TT) tile[f] = tv[k];
    if constexpr (GRAD)
      if (f < TT) ztile[f] = zl[k];
  }
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
      if constexpr (GRAD) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const double wp = lane_d(gwp, dl[g]), wq = lane_d(gwq, dl[g]);
          const int qg = __builtin_amdgcn_readlane(gqi, dl[g]);
          double cp = 0.0, dp = 0.0;
#pragma unroll
          for (int k = 0; k < EPT; ++k) {
            const double2 z = zf(k);
            cp += gcross(v[g][k], z);
            dp += gdot(v[g][k], z);
          }
#pragma unroll
          for (int qq = 0; qq < QC; ++qq)
            if (qq == qg) {  // uniform
              ga->p[qq] += wp * cp;
              ga->q[qq] += wq * dp;
            }
        }
      }
    }
  } else {
    // One entry per thread, or the largest blocks: the directions one at a
    // time under uniform branches (measured faster there than the table).
    // GRAD: the integrand weights (wp, wq) of subsystem q as in the table.
    auto direction = [&](double2 c, int64_t shift, int q, double wp, double wq) {
      if constexpr (!GRAD) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) cmac(acc[k], c, X[offs[k] + shift]);
        return;
      }
      double2 v[EPT];
#pragma unroll
      for (int k = 0; k < EPT; ++k) v[k] = X[offs[k] + shift];
#pragma unroll
      for (int k = 0; k < EPT; ++k) cmac(acc[k], c, v[k]);
      if constexpr (GRAD) {
        double cp = 0.0, dp = 0.0;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const double2 z = zf(k);
          cp += gcross(v[k], z);
          dp += gdot(v[k], z);
        }
        ga->p[q] += wp * cp;
        ga->q[q] += wq * dp;
      }
    };
#pragma unroll
    for (int q = 0; q < ER; ++q) {
      const int n = ne[q];
      const int64_t sN = (int64_t)S.stride[q] * N;
      if (n + 1 < NL)
        direction(ctl_coef<DIR_RP, ADJ>(da[q], db[q], sqrt_small<NL>(n + 1)), sN, q, sqrt_small<NL>(n + 1),
                  -sqrt_small<NL>(n + 1));
      if (n > 0) direction(ctl_coef<DIR_RM, ADJ>(da[q], db[q], sqrt_small<NL>(n)), -sN, q, sqrt_small<NL>(n),
                           sqrt_small<NL>(n));
    }
#pragma unroll
    for (int q = 0; q < EC; ++q) {
      const int m = me[q];
      const int64_t s1 = S.stride[q];
      if (m + 1 < NL)
        direction(ctl_coef<DIR_CP, ADJ>(da[q], db[q], sqrt_small<NL>(m + 1)), s1, q, -sqrt_small<NL>(m + 1),
                  -sqrt_small<NL>(m + 1));
      if (m > 0) direction(ctl_coef<DIR_CM, ADJ>(da[q], db[q], sqrt_small<NL>(m)), -s1, q, -sqrt_small<NL>(m),
                           sqrt_small<NL>(m));
    }
#pragma unroll
    for (int q = 0; q < (ER < EC ? ER : EC); ++q) {
      const int n = ne[q], m = me[q];
      const bool jr = !ADJ ? (n + 1 < NL && m + 1 < NL) : (n > 0 && m > 0);
      if (jr) {
        const double cj = !ADJ ? S.g1[q] * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1)
                               : S.g1[q] * sqrt_small<NL>(n) * sqrt_small<NL>(m);
        const int64_t sj = (int64_t)S.stride[q] * N + S.stride[q];
        direction(make_double2(cj, 0.0), !ADJ ? sj : -sj, q, 0.0, 0.0);
      }
    }
  }
  __syncthreads();
  // Internal terms (LDS), the diagonal data and the output, entry by entry.
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
    Entry en;
    en.e = b * N2 + offs[k];
    en.f = f;
    en.acc = ac;
    en.own = tile[f];
    en.gam = gam;
    en.dE = Es[i] - Es[j];
    out(en);
  }
  // GRAD: the integrand terms of the internal digits, in a pass of their own
  // over the LDS block (the stencil's registers are free by now).
  if constexpr (GRAD) {
#pragma unroll 1
    for (int k = 0; k < EPT; ++k) {
      const int f = tid + k * BLOCK;
      if (f >= TT) continue;
      const double2 z = ztile[f];
      int ra = f / TC, rc = f - (f / TC) * TC;
#pragma unroll
      for (int q = QC - 1; q >= 0; --q) {
        const int st = S.stride[q];
        if (q >= ER) {
          const int n = ra % NL;
          ra /= NL;
          const bool rp = n + 1 < NL, rm = n > 0;
          const double2 vp = tile[f + (rp ? st * TC : 0)], vm = tile[f - (rm ? st * TC : 0)];
          const double wp = rp ? sqrt_small<NL>(n + 1) : 0.0, wm = sqrt_small<NL>(n);
          ga->p[q] += wp * gcross(vp, z) + wm * gcross(vm, z);
          ga->q[q] += -wp * gdot(vp, z) + wm * gdot(vm, z);
        }
        if (q >= EC) {
          const int m = rc % NL;
          rc /= NL;
          const bool cp = m + 1 < NL, cm = m > 0;
          const double2 vp = tile[f + (cp ? st : 0)], vm = tile[f - (cm ? st : 0)];
          const double wp = cp ? sqrt_small<NL>(m + 1) : 0.0, wm = sqrt_small<NL>(m);
          ga->p[q] += -wp * gcross(vp, z) - wm * gcross(vm, z);
          ga->q[q] += -wp * gdot(vp, z) + wm * gdot(vm, z);
        }
      }
    }
  }
}

}  // namespace tile
}  // namespace lbx

// Instantiated block shapes (NL, Q, KR, KC, threads per block); the first
// listed for a (NL, Q) is the default.  Blocks of up to 2187 entries run 256
// threads, so that several fit on one compute unit.
#ifdef LBX_ONE_SHAPE
#define LBX_TILE_SHAPES(X) X(3, 8, 3, 4, 256) X(3, 8, 4, 2, 256)
#else
#define LBX_TILE_SHAPES(X)                                                                    \
  X(3, 8, 4, 4, 512) X(3, 8, 4, 3, 256) X(3, 8, 3, 4, 256) X(3, 8, 4, 2, 256)                  \
  X(3, 8, 3, 3, 256) X(3, 8, 3, 2, 256) X(3, 8, 2, 3, 256)                                     \
  X(3, 7, 4, 4, 512) X(3, 7, 4, 3, 256) X(3, 7, 3, 3, 256) X(3, 6, 4, 4, 512)                  \
  X(3, 6, 4, 3, 256) X(3, 5, 3, 3, 256) X(3, 5, 3, 2, 256) X(3, 5, 2, 3, 256)                  \
  X(2, 9, 6, 6, 512) X(2, 10, 6, 6, 512) X(2, 11, 6, 6, 512) X(2, 12, 6, 6, 512)               \
  X(4, 5, 3, 3, 512) X(4, 6, 3, 3, 512)
#endif
