// Block-tiled streaming kernels for large systems of equal-level subsystems
// (the eight-qutrit ring is the design case): lindblad_apply (tile_kernel)
// and the gradient integrands of one step (tile_grad_kernel) of a single
// streamed system whose subsystems all have NL levels, in one of the
// LBX_TILE_SHAPES, and the multi-pass apply (pass_kernel, LB_OPT_TILE 2).
// The stage sweeps of the implicit-midpoint steps use the same tiles inside
// the persistent step kernels of kernels_step.hip.
#include <hip/hip_runtime.h>

#include "lbx_host.hpp"
#include "tile_unit.hpp"

namespace lbx {

constexpr int TILE_BLOCK = 512;  // threads of the multi-pass kernels

using tile::cmac;
using tile::ctl_coef;
using tile::DIR_CM;
using tile::DIR_CP;
using tile::DIR_RM;
using tile::DIR_RP;
using tile::ipow;
using tile::sqrt_small;
using tile::uniform;

// y = M x (or M^+ x) for B states, one unit per workgroup (tile_unit.hpp);
// blocks are remapped so that each XCD (blocks are dealt to the 8 XCDs
// round-robin) walks a contiguous band of units.  Every wavefront forms the
// controls, lane q holding d_q, before the block's loads, so that no loaded
// value is live across the evaluation.
template <int NL, int QC, int KR, int KC, bool ADJ, int BLOCK>
__global__ __launch_bounds__(BLOCK) void tile_kernel(const SysDev *__restrict__ sysv, int sys, int64_t nblocks,
                                                     const double *__restrict__ Etab,
                                                     const double *__restrict__ alpha,
                                                     const double *__restrict__ carrier, double t,
                                                     const double2 *__restrict__ x, double2 *__restrict__ y) {
  extern __shared__ double2 tileb[];
  const SysDev &S = sysv[sys];
  const int64_t per = (nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= nblocks) return;
  const int lane = threadIdx.x & 63;
  double2 dv = make_double2(0.0, 0.0);
  if (lane < QC) dv = control_value(S, alpha, carrier + S.carrier_off, lane, t);
  double da[QC], db[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    da[q] = tile::lane_d(dv.x, q);
    db[q] = tile::lane_d(dv.y, q);
  }
  tile::tile_unit<NL, QC, KR, KC, ADJ, BLOCK>(S, lb, x, tileb, da, db, Etab + S.tab_off, false,
                                              [&](const tile::Entry &en) {
                                                y[en.e] = cadd(en.acc, cmul(diag_coef(en.gam, en.dE, ADJ), en.own));
                                              });
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
  extern __shared__ double2 tls[];
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
    if (f < TT) tls[f] = v;
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
        const double2 vp = tls[f + (rp ? st * TC : 0)], vm = tls[f - (rm ? st * TC : 0)];
        const double wp = rp ? sqrt_small<NL>(n + 1) : 0.0, wm = sqrt_small<NL>(n);
        gp[q] += wp * cross2(vp, z[k]) + wm * cross2(vm, z[k]);
        gq[q] += -wp * dot2(vp, z[k]) + wm * dot2(vm, z[k]);
      }
      if (q >= EC) {
        const int m = rc % NL;
        rc /= NL;
        const bool cp = m + 1 < NL, cm = m > 0;
        const double2 vp = tls[f + (cp ? st : 0)], vm = tls[f - (cm ? st : 0)];
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
  extern __shared__ double2 tls[];
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
      if (f < TT) tls[f] = tv[k];
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
      cmac(ac, ctl_coef<DIR_RP, ADJ>(da[q], db[q], rp ? sqrt_small<NL>(n + 1) : 0.0), tls[f + (rp ? sr : 0)]);
      cmac(ac, ctl_coef<DIR_RM, ADJ>(da[q], db[q], sqrt_small<NL>(n)), tls[f - (rm ? sr : 0)]);
      cmac(ac, ctl_coef<DIR_CP, ADJ>(da[q], db[q], cp ? sqrt_small<NL>(m + 1) : 0.0), tls[f + (cp ? sc : 0)]);
      cmac(ac, ctl_coef<DIR_CM, ADJ>(da[q], db[q], sqrt_small<NL>(m)), tls[f - (cm ? sc : 0)]);
      const bool jr = !ADJ ? (rp && cp) : (rm && cm);
      const double cj = !jr ? 0.0
                            : !ADJ ? S.g1[q] * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1)
                                   : S.g1[q] * sqrt_small<NL>(n) * sqrt_small<NL>(m);
      const double2 vj = tls[f + (!jr ? 0 : !ADJ ? sr + sc : -(sr + sc))];
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
      out[e] = cadd(ac, cmul(D, tls[f]));
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
  if (S.njc > 0) return 0;
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

// Block shapes: KR row digits and KC column digits inside a block
// (LBX_TILE_SHAPES in tile_unit.hpp).  The default is the shape listed first
// for the system (the largest square block, at most 6561 entries); the
// LB_OPT_TILE_KI option selects another instantiated shape (10*KR + KC).
int tile_ki(const lb_plan *p, int sys, int ki_opt) {
  const SysDev &S = p->sys[sys];
  if (S.njc > 0) return 0;  // the coupling runs on the generic kernels
  if (ki_opt >= LB_SPLIT_BASE) {  // two-pass sweep and apply (any levels)
    SplitGeo g;
    return split_geo(p, sys, ki_opt, &g) ? ki_opt : 0;
  }
  const int nl = S.nlev[0];
  for (int q = 1; q < S.Q; ++q)
    if (S.nlev[q] != nl) return 0;
  int first = 0;
#define X(A, B, R, C, T)                                           \
  if (nl == A && S.Q == B) {                                       \
    if (!first) first = 10 * R + C;                                \
    if (ki_opt == 10 * R + C) return 10 * R + C;                   \
  }
  LBX_TILE_SHAPES(X)
#undef X
  return first;
}

template <int NL, int QC, int KR, int KC, int BLOCK, bool ADJ>
static int tile_launch(const lb_plan *p, int sys, int B, const double *alpha, double t, const double2 *x,
                       double2 *y, hipStream_t st) {
  using Sh = tile::Shape<NL, QC, KR, KC, BLOCK>;
  const size_t shmem = Sh::lds_bytes();
  auto kern = tile_kernel<NL, QC, KR, KC, ADJ, BLOCK>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const int64_t nblocks = tile::tile_units(p->sys[sys].N, Sh::TR, Sh::TC, B);
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(BLOCK), shmem, st, p->d_sys, sys, nblocks, p->d_E, alpha,
                     p->d_carrier, t, x, y);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

template <int NL, int QC, int KR, int KC, int BLOCK>
static int tile_grad_launch(const lb_plan *p, int sys, int B, const double2 *zh, const double2 *q0,
                            const double2 *q1, double *gpart, int64_t *rows, hipStream_t st) {
  using Sh = tile::Shape<NL, QC, KR, KC, BLOCK>;
  const size_t shmem = Sh::lds_bytes();
  auto kern = tile_grad_kernel<NL, QC, KR, KC, BLOCK>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const int64_t nblocks = tile::tile_units(p->sys[sys].N, Sh::TR, Sh::TC, B);
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(BLOCK), shmem, st, p->d_sys, sys, nblocks, zh, q0,
                     q1, gpart);
  LBX_HIP(hipGetLastError());
  *rows = nblocks;
  return LB_OK;
}

// Gradient integrands of one step for a system on the block-tiled path, in
// block shape k.  *rows receives the number of partial rows.
int launch_tile_grad(const lb_plan *p, int sys, int B, int k, const double2 *zh, const double2 *q0,
                     const double2 *q1, double *gpart, int64_t *rows, hipStream_t st) {
  *rows = 0;
  if (B == 0) return LB_OK;
  if (k >= LB_SPLIT_BASE) k = tile_ki(p, sys, 0);  // the two-pass sweeps keep the block-tiled integrands
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0];
#define X(A, Bq, R, C, T) \
  if (nl == A && S.Q == Bq && k == 10 * R + C) return tile_grad_launch<A, Bq, R, C, T>(p, sys, B, zh, q0, q1, gpart, rows, st);
  LBX_TILE_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "system not eligible for the tiled gradient kernel");
}

int64_t tile_grad_rows(const lb_plan *p, int sys, int B, int k) {
  const SysDev &S = p->sys[sys];
  if (k >= LB_SPLIT_BASE) k = tile_ki(p, sys, 0);
  if (!k) return 0;
  int tr = 1, tc = 1;
  for (int i = 0; i < k / 10; ++i) tr *= S.nlev[0];
  for (int i = 0; i < k % 10; ++i) tc *= S.nlev[0];
  return (int64_t)B * (S.N / tr) * (S.N / tc);
}

int launch_tile_apply(const lb_plan *p, int sys, int B, bool adj, const double *alpha, double t, const double2 *x,
                      double2 *y, int tile_opt, int ki_opt, hipStream_t st) {
  if (B == 0) return LB_OK;
  if (ki_opt >= LB_SPLIT_BASE) {
    SplitGeo g;
    if (split_geo(p, sys, ki_opt, &g)) return launch_split_apply(p, sys, B, adj, t, alpha, x, y, g, st);
  }
  if (tile_opt == 2 && split_kl(p, sys))
    return launch_split(p, sys, B, 0, adj, alpha, t, nullptr, 0, x, nullptr, y, nullptr, st);
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0], k = tile_ki(p, sys, ki_opt);
#define X(A, Bq, R, C, T)                                                                     \
  if (nl == A && S.Q == Bq && k == 10 * R + C)                                                \
    return adj ? tile_launch<A, Bq, R, C, T, true>(p, sys, B, alpha, t, x, y, st)             \
               : tile_launch<A, Bq, R, C, T, false>(p, sys, B, alpha, t, x, y, st);
  LBX_TILE_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "system not eligible for the tiled kernels");
}

}  // namespace lbx
