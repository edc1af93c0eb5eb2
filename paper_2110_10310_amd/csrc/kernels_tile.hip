// Row-tiled streaming kernels for large systems of equal-level subsystems.
//
// Block-tiled streaming kernels for large systems of equal-level subsystems
// (the eight-qutrit ring is the design case).  Used for lindblad_apply and
// for the stage-solve sweeps of a single streamed system when every
// subsystem has the same number of levels NL and the shape is one of
// LBX_TILE_SHAPES.  See tile_kernel for the tiling.
#include <hip/hip_runtime.h>

#include "lbx_host.hpp"

namespace lbx {

constexpr int TILE_BLOCK = 512;

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

// Contribution of one subsystem with row digit n, column digit m, control
// (a, b) = (Re d, Im d) and the five neighbour values; see `offdiag`.
template <int NL, bool ADJ>
__device__ __forceinline__ void tile_term(int n, int m, double g1, double g2, double a, double b,
                                          double2 vrp, double2 vrm, double2 vcp, double2 vcm,
                                          double2 vj, double2 &acc, double &gam) {
  const bool rp = n + 1 < NL, rm = n > 0, cp = m + 1 < NL, cm = m > 0;
  const double dnm = (double)(n - m);
  gam += 0.5 * (g1 * (double)(n + m) + g2 * dnm * dnm);
  const double arp = rp ? sqrt_small<NL>(n + 1) : 0.0;
  const double arm = sqrt_small<NL>(n);
  const double acp = cp ? sqrt_small<NL>(m + 1) : 0.0;
  const double acm = sqrt_small<NL>(m);
  const double2 U = make_double2(arp * vrp.x - acm * vcm.x, arp * vrp.y - acm * vcm.y);
  const double2 V = make_double2(arm * vrm.x - acp * vcp.x, arm * vrm.y - acp * vcp.y);
  const double2 Sm = cadd(U, V), Dv = csub(U, V);
  const double cr = a * Sm.y + b * Dv.x;
  const double ci = -a * Sm.x + b * Dv.y;
  const double cj = !ADJ ? ((rp && cp) ? g1 * sqrt_small<NL>(n + 1) * sqrt_small<NL>(m + 1) : 0.0)
                         : ((rm && cm) ? g1 * sqrt_small<NL>(n) * sqrt_small<NL>(m) : 0.0);
  if (!ADJ) {
    acc.x += cr + cj * vj.x;
    acc.y += ci + cj * vj.y;
  } else {
    acc.x += -cr + cj * vj.x;
    acc.y += -ci + cj * vj.y;
  }
}

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

__device__ __forceinline__ double uniform(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

}  // namespace

// MODE 0: y = M x (or M^+ x).  MODE 1: out = q + delta.  MODE 2: out = q + 2 delta,
// delta = w (h D q + h O zin) as in sweep_kernel.
//
// A workgroup owns one TR x TC block of a state, TR = NL^KR rows and
// TC = NL^KC columns: the KR (KC) least significant digits of the row
// (column) index vary and the others are fixed.  The block is staged in LDS,
// so every neighbour along an internal digit (row or column ladder shift, or
// decay jump of a subsystem internal in both) is an LDS read.  Neighbours
// along the external digits are global loads, all issued before any is used;
// their weights depend only on the fixed digits (uniform over the
// workgroup), and a missing one reads the entry itself with a zero weight.
// Blocks are remapped so that each XCD (blocks are dealt to the 8 XCDs
// round-robin) walks a contiguous band of block rows.
template <int NL, int QC, int KR, int KC, bool ADJ, int MODE>
__global__ __launch_bounds__(TILE_BLOCK) void tile_kernel(
    const SysDev *__restrict__ sysv, int sys, int64_t nblocks, const double *__restrict__ Etab,
    const double *__restrict__ alpha, const double *__restrict__ carrier, double t,
    const double2 *__restrict__ ctab, int jstep, const double2 *__restrict__ zin,
    const double2 *__restrict__ qin, double2 *__restrict__ out) {
  extern __shared__ double2 tile[];
  __shared__ double2 dqs[QC];
  constexpr int ER = QC - KR, EC = QC - KC;  // external row / column digits
  constexpr int TR = ipow(NL, KR), TC = ipow(NL, KC);
  const SysDev &S = sysv[sys];
  const int N = S.N;
  const int NBR = N / TR, NBC = N / TC;
  const int64_t N2 = S.N2;
  const int tid = threadIdx.x;
  const int64_t per = (nblocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= nblocks) return;
  if (tid < QC)
    dqs[tid] = ctab ? ctab[S.ctab_off + (int64_t)jstep * QC + tid]
                    : control_value(S, alpha, carrier + S.carrier_off, tid, t);
  const int64_t b = lb / ((int64_t)NBR * NBC);
  const int rem = (int)(lb - b * NBR * NBC);
  const int bi = rem / NBC, bj = rem - (rem / NBC) * NBC;
  const double2 *X = zin + b * N2;
  const int64_t base = (int64_t)bi * TR * N + (int64_t)bj * TC;
  for (int f = tid; f < TR * TC; f += TILE_BLOCK) {
    const int a = f / TC, c = f - (f / TC) * TC;
    tile[f] = X[base + (int64_t)a * N + c];
  }
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
  const double h = S.h;
  const double *Es = Etab + S.tab_off;
  __syncthreads();
  double da[QC], db[QC];
#pragma unroll
  for (int q = 0; q < QC; ++q) {
    da[q] = uniform(dqs[q].x);
    db[q] = uniform(dqs[q].y);
  }
  for (int f = tid; f < TR * TC; f += TILE_BLOCK) {
    const int a = f / TC, c = f - (f / TC) * TC;
    const int64_t e0 = base + (int64_t)a * N + c;
    // all digits of this entry
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
    // global neighbour loads first
    double2 gr[ER > 0 ? 2 * ER : 1], gc[EC > 0 ? 2 * EC : 1], gj[QC];
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int n = nd[q], m = md[q];
      const int64_t s1 = S.stride[q];
      const int64_t sN = s1 * N;
      const bool rp = n + 1 < NL, rm = n > 0, cp = m + 1 < NL, cm = m > 0;
      if (q < ER) {
        gr[2 * q] = X[e0 + (rp ? sN : 0)];
        gr[2 * q + 1] = X[e0 - (rm ? sN : 0)];
      }
      if (q < EC) {
        gc[2 * q] = X[e0 + (cp ? s1 : 0)];
        gc[2 * q + 1] = X[e0 - (cm ? s1 : 0)];
      }
      if (q < ER || q < EC) {
        if (!ADJ) gj[q] = X[e0 + ((rp && cp) ? sN + s1 : 0)];
        else gj[q] = X[e0 - ((rm && cm) ? sN + s1 : 0)];
      }
    }
    double2 acc = make_double2(0.0, 0.0);
    double gam = 0.0;
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      const int n = nd[q], m = md[q];
      const bool rp = n + 1 < NL, rm = n > 0, cp = m + 1 < NL, cm = m > 0;
      const int st = S.stride[q];
      double2 vrp, vrm, vcp, vcm, vj;
      if (q < ER) {
        vrp = gr[2 * q];
        vrm = gr[2 * q + 1];
      } else {  // internal row digit: a row shift of st is st*TC entries in the block
        vrp = tile[f + (rp ? st * TC : 0)];
        vrm = tile[f - (rm ? st * TC : 0)];
      }
      if (q < EC) {
        vcp = gc[2 * q];
        vcm = gc[2 * q + 1];
      } else {
        vcp = tile[f + (cp ? st : 0)];
        vcm = tile[f - (cm ? st : 0)];
      }
      if (q < ER || q < EC) {
        vj = gj[q];
      } else if (!ADJ) {
        vj = tile[f + ((rp && cp) ? st * TC + st : 0)];
      } else {
        vj = tile[f - ((rm && cm) ? st * TC + st : 0)];
      }
      tile_term<NL, ADJ>(n, m, S.g1[q], S.g2[q], da[q], db[q], vrp, vrm, vcp, vcm, vj, acc, gam);
    }
    const int i = bi * TR + a, j = bj * TC + c;
    const double dE = Es[i] - Es[j];
    const double2 D = diag_coef(gam, dE, ADJ);
    const int64_t e = b * N2 + e0;
    if (MODE == 0) {
      out[e] = cadd(acc, cmul(D, tile[f]));
    } else {
      const double2 qv = qin[e];
      const double2 w = stage_weight(h, gam, dE, ADJ);
      const double2 hdq = cscale(h, cmul(D, qv));
      const double2 dn = cmul(w, make_double2(hdq.x + h * acc.x, hdq.y + h * acc.y));
      out[e] = MODE == 2 ? make_double2(qv.x + 2.0 * dn.x, qv.y + 2.0 * dn.y) : cadd(qv, dn);
    }
  }
}

// Block shapes: KR row digits and KC column digits inside a block.  The
// default is the square block with the most entries up to 6561; the plan's
// LB_OPT_TILE_KI selects another instantiated shape (encoded 10*KR + KC).
constexpr int TILE_MAX = 6561;

template <int NL, int QC, int KR, int KC, bool ADJ, int MODE>
static int tile_launch(const lb_plan *p, int sys, int B, const double *alpha, double t,
                       const double2 *ctab, int j, const double2 *zin, const double2 *qin,
                       double2 *out, hipStream_t st) {
  constexpr int TR = ipow(NL, KR), TC = ipow(NL, KC);
  const int N = p->sys[sys].N;
  const size_t shmem = (size_t)TR * TC * sizeof(double2);
  auto kern = tile_kernel<NL, QC, KR, KC, ADJ, MODE>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  const int64_t nblocks = (int64_t)B * (N / TR) * (N / TC);
  const int64_t grid = ((nblocks + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(TILE_BLOCK), shmem, st, p->d_sys, sys, nblocks,
                     p->d_E, alpha, p->d_carrier, t, ctab, j, zin, qin, out);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

template <int NL, int QC, int KR, int KC>
static int tile_modes(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha,
                      double t, const double2 *ctab, int j, const double2 *zin, const double2 *qin,
                      double2 *out, hipStream_t st) {
  if (adj) {
    if (mode == 0) return tile_launch<NL, QC, KR, KC, true, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, st);
    if (mode == 1) return tile_launch<NL, QC, KR, KC, true, 1>(p, sys, B, alpha, t, ctab, j, zin, qin, out, st);
    return tile_launch<NL, QC, KR, KC, true, 2>(p, sys, B, alpha, t, ctab, j, zin, qin, out, st);
  }
  if (mode == 0) return tile_launch<NL, QC, KR, KC, false, 0>(p, sys, B, alpha, t, ctab, j, zin, qin, out, st);
  if (mode == 1) return tile_launch<NL, QC, KR, KC, false, 1>(p, sys, B, alpha, t, ctab, j, zin, qin, out, st);
  return tile_launch<NL, QC, KR, KC, false, 2>(p, sys, B, alpha, t, ctab, j, zin, qin, out, st);
}

// Instantiated shapes (NL, Q, KR, KC); the first listed for a (NL, Q) is the default.
#define LBX_TILE_SHAPES(X)                                                                    \
  X(3, 8, 4, 4) X(3, 8, 4, 3) X(3, 8, 3, 4) X(3, 8, 4, 2) X(3, 8, 3, 3)                          \
  X(3, 7, 4, 4) X(3, 7, 4, 3) X(3, 6, 4, 4) X(3, 6, 4, 3)                                       \
  X(2, 9, 6, 6) X(2, 10, 6, 6) X(2, 11, 6, 6) X(2, 12, 6, 6) X(4, 5, 3, 3) X(4, 6, 3, 3)

int tile_ki(const lb_plan *p, int sys) {
  const SysDev &S = p->sys[sys];
  const int nl = S.nlev[0];
  for (int q = 1; q < S.Q; ++q)
    if (S.nlev[q] != nl) return 0;
  int first = 0;
#define X(A, B, R, C)                                              \
  if (nl == A && S.Q == B) {                                       \
    if (!first) first = 10 * R + C;                                \
    if (p->tile_ki == 10 * R + C) return 10 * R + C;               \
  }
  LBX_TILE_SHAPES(X)
#undef X
  return first;
}

int tile_nl(const lb_plan *p, int sys) { return tile_ki(p, sys) > 0 ? p->sys[sys].nlev[0] : 0; }

int launch_tile(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha, double t,
                const double2 *ctab, int j, const double2 *zin, const double2 *qin, double2 *out,
                hipStream_t st) {
  if (B == 0) return LB_OK;
  const SysDev &S = p->sys[sys];
  const int nl = tile_nl(p, sys), k = tile_ki(p, sys);
#define X(A, Bq, R, C) \
  if (nl == A && S.Q == Bq && k == 10 * R + C) return tile_modes<A, Bq, R, C>(p, sys, B, mode, adj, alpha, t, ctab, j, zin, qin, out, st);
  LBX_TILE_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "system not eligible for the tiled kernels");
}

}  // namespace lbx
