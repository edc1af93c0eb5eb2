// LDS-resident persistent kernels specialised on the number of subsystems.
//
// Same algorithm and memory layout as the generic kernels of
// kernels_lds.hip (one workgroup per state, stage iterate in two LDS
// buffers, delta-form fixed-point sweeps), for systems with few subsystems
// and at most four (entry, subsystem) pairs per thread.  Everything that does
// not change over the time loop is computed once per entry and kept in
// registers: the ladder weights sqrt(n), sqrt(n+1), sqrt(m), sqrt(m+1) with
// the boundary cases folded in as zeros, the decay-jump weight, and the LDS
// offsets of every neighbour (the entry itself where a neighbour does not
// exist, with a zero weight).  A sweep is then LDS reads and FP64 FMAs only;
// the per-step control values come through scalar loads.  The adjoint
// reduces its per-step gradient integrands over 16-lane DPP rows.
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

template <int BLOCK, int EPT, int QC>
__global__ __launch_bounds__(BLOCK) void lds_forward_fast_kernel(
    const SysDev *__restrict__ sysv, const LdsItem *__restrict__ items,
    const double *__restrict__ Etab, const uint64_t *__restrict__ desc,
    const double2 *__restrict__ ctab, const int32_t *__restrict__ ktab, int NT,
    const double2 *__restrict__ rho0, double2 *__restrict__ rhoT, double2 *__restrict__ states) {
  extern __shared__ double2 zbuf[];
  const LdsItem it = items[blockIdx.x];
  const SysDev &S = sysv[it.sys];
  const int tid = threadIdx.x;
  const int N = S.N;
  const int N2 = (int)S.N2;
  const double h = S.h;
  const double2 *cq = ctab + S.ctab_off;
  const int32_t *kt = ktab + (int64_t)it.sys * NT * 2;

  double2 qv[EPT], wv[EPT], hd[EPT], dn[EPT];
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
    if (states && ok[k]) states[it.st_off + e] = qv[k];
  }
  // Two LDS stage buffers; selected by value (not through a pointer array)
  // so that every access stays an LDS instruction.
  double2 *const zb0 = zbuf, *const zb1 = zbuf + N2;
  int cb = 0;
  for (int j = 0; j < NT; ++j) {
    double2 dq[QC];
#pragma unroll
    for (int q = 0; q < QC; ++q) dq[q] = cq[(int64_t)j * QC + q];
    const int K = kt[2 * j];
    double2 hdq[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      hdq[k] = cmul(hd[k], qv[k]);
      if (ok[k]) (cb ? zb1 : zb0)[ee[k]] = cadd(qv[k], cmul(wv[k], hdq[k]));
    }
    __syncthreads();
    for (int kk = 0; kk < K; ++kk) {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<false, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
      }
      if (kk + 1 < K) {
        double2 *dst = (cb ? zb0 : zb1);
#pragma unroll
        for (int k = 0; k < EPT; ++k)
          if (ok[k]) dst[ee[k]] = cadd(qv[k], dn[k]);
        __syncthreads();
        cb ^= 1;
      }
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      qv[k] = make_double2(qv[k].x + 2.0 * dn[k].x, qv[k].y + 2.0 * dn[k].y);
      if (states && ok[k]) states[it.st_off + (int64_t)(j + 1) * N2 + ee[k]] = qv[k];
    }
    cb ^= 1;
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k)
    if (ok[k]) rhoT[it.off + ee[k]] = qv[k];
}

template <int BLOCK, int EPT, int QC>
__global__ __launch_bounds__(BLOCK) void lds_adjoint_fast_kernel(
    const SysDev *__restrict__ sysv, const LdsItem *__restrict__ items,
    const double *__restrict__ Etab, const uint64_t *__restrict__ desc,
    const double2 *__restrict__ ctab, const int32_t *__restrict__ ktab, int NT, int kind,
    const double2 *__restrict__ rhotar, const double2 *__restrict__ states,
    double *__restrict__ gpart) {
  extern __shared__ double2 zbuf[];
  constexpr int ROWS = BLOCK / 16;
  const LdsItem it = items[blockIdx.x];
  const SysDev &S = sysv[it.sys];
  const int tid = threadIdx.x;
  const int N = S.N;
  const int N2 = (int)S.N2;
  const double h = S.h;
  const double2 *cq = ctab + S.ctab_off;
  const int32_t *kt = ktab + (int64_t)it.sys * NT * 2;
  const double2 *hist = states + it.st_off;

  double2 qh[EPT], wv[EPT], hd[EPT], dn[EPT], qn[EPT];
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
    qn[k] = ok[k] ? hist[(int64_t)NT * N2 + ee[k]] : make_double2(0.0, 0.0);
    const double2 t = ok[k] ? rhotar[it.off + ee[k]] : make_double2(0.0, 0.0);
    qh[k] = kind == LB_J_FROB ? cscale(it.wterm, csub(qn[k], t)) : cscale(-it.wterm, t);
    dn[k] = make_double2(0.0, 0.0);
  }
  // Two LDS stage buffers; selected by value (not through a pointer array)
  // so that every access stays an LDS instruction.
  double2 *const zb0 = zbuf, *const zb1 = zbuf + N2;
  int cb = 0;
  for (int j = NT - 1; j >= 0; --j) {
    double2 dq[QC];
#pragma unroll
    for (int q = 0; q < QC; ++q) dq[q] = cq[(int64_t)j * QC + q];
    const int K = kt[2 * j];
    // (I - h M^+) zh = qh^{j+1} (App. B eq. linsystem_adjoint), zh = qh + delta.
    double2 hdq[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      hdq[k] = cmul(hd[k], qh[k]);
      if (ok[k]) (cb ? zb1 : zb0)[ee[k]] = cadd(qh[k], cmul(wv[k], hdq[k]));
    }
    // Forward state q^j, consumed after the sweeps so that its load overlaps them.
    double2 qj[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) qj[k] = ok[k] ? hist[(int64_t)j * N2 + ee[k]] : make_double2(0.0, 0.0);
    __syncthreads();
    for (int kk = 0; kk < K; ++kk) {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const double2 acc = offdiag_nb<true, QC>(nb[k], dq, src);
        dn[k] = cmul(wv[k], make_double2(hdq[k].x + h * acc.x, hdq[k].y + h * acc.y));
      }
      if (kk + 1 < K) {
        double2 *dst = (cb ? zb0 : zb1);
#pragma unroll
        for (int k = 0; k < EPT; ++k)
          if (ok[k]) dst[ee[k]] = cadd(qh[k], dn[k]);
        __syncthreads();
        cb ^= 1;
      }
    }
    // Gradient integrands (see grad_term in lbx_device.hpp) need zh at neighbours.
    double2 *zhb = (cb ? zb0 : zb1);
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      if (ok[k]) zhb[ee[k]] = cadd(qh[k], dn[k]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QC; ++q) {
      double gp = 0.0, gq = 0.0;
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        if (ok[k]) {
          const double2 z = make_double2(0.5 * (qj[k].x + qn[k].x), 0.5 * (qj[k].y + qn[k].y));
          double2 U, V;
          uv(nb[k][q], zhb, U, V);
          const double2 Sm = cadd(U, V), Dv = csub(U, V);
          gp += Sm.x * z.y - Sm.y * z.x;
          gq -= Dv.x * z.x + Dv.y * z.y;
        }
      }
      gp = row16_sum(gp);
      gq = row16_sum(gq);
      if ((tid & 15) == 15) {
        double *dstp = gpart + it.gp_off + ((int64_t)j * ROWS + (tid >> 4)) * 2 * QC + 2 * q;
        dstp[0] = gp;
        dstp[1] = gq;
      }
    }
    // qh^j = qh^{j+1} + dt M^+ zh = qh^{j+1} + 2 delta.
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      qh[k] = make_double2(qh[k].x + 2.0 * dn[k].x, qh[k].y + 2.0 * dn[k].y);
      qn[k] = qj[k];
    }
  }
}

// Shapes with a specialised kernel.  Workgroups of 1024 threads leave 128
// VGPRs per thread, which bounds the register-resident stencil data there.
bool lds_fast_ok(int block, int ept, int Q) {
  if (Q < 1 || Q > 4) return false;
  if (ept == 1) return block <= 512 || Q <= 3;
  return block == 1024 && ept == 2 && Q == 1;
}

template <int BLOCK, int EPT, int QC>
static int fwd_t(const lb_plan *p, const LdsItem *d_items, int nitems, const double2 *ctab,
                 const int32_t *ktab, const double2 *rho0, double2 *rhoT, double2 *states,
                 hipStream_t st) {
  const size_t shmem = (size_t)2 * BLOCK * EPT * sizeof(double2);
  auto kern = lds_forward_fast_kernel<BLOCK, EPT, QC>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(BLOCK), shmem, st, p->d_sys, d_items, p->d_E, p->d_desc,
                     ctab, ktab, p->NT, rho0, rhoT, states);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

template <int BLOCK, int EPT, int QC>
static int adj_t(const lb_plan *p, const LdsItem *d_items, int nitems, int kind, const double2 *ctab,
                 const int32_t *ktab, const double2 *rhotar, const double2 *states, double *gpart,
                 hipStream_t st) {
  const size_t shmem = (size_t)2 * BLOCK * EPT * sizeof(double2);
  auto kern = lds_adjoint_fast_kernel<BLOCK, EPT, QC>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem));
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(BLOCK), shmem, st, p->d_sys, d_items, p->d_E, p->d_desc,
                     ctab, ktab, p->NT, kind, rhotar, states, gpart);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

#define LBX_FAST_SHAPES(X)                                                                  \
  X(64, 1, 1) X(64, 1, 2) X(64, 1, 3) X(64, 1, 4) X(128, 1, 1) X(128, 1, 2) X(128, 1, 3)    \
  X(128, 1, 4) X(256, 1, 1) X(256, 1, 2) X(256, 1, 3) X(256, 1, 4) X(512, 1, 1) X(512, 1, 2) \
  X(512, 1, 3) X(512, 1, 4) X(1024, 1, 1) X(1024, 1, 2) X(1024, 1, 3) X(1024, 2, 1)

int launch_lds_forward_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, const double2 *ctab, const int32_t *ktab, const double2 *rho0,
                            double2 *rhoT, double2 *states, hipStream_t st) {
  if (nitems == 0) return LB_OK;
#define X(B, E, C) \
  if (block == B && ept == E && Q == C) return fwd_t<B, E, C>(p, d_items, nitems, ctab, ktab, rho0, rhoT, states, st);
  LBX_FAST_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "no specialised LDS-resident kernel for this shape");
}

int launch_lds_adjoint_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, int kind, const double2 *ctab, const int32_t *ktab,
                            const double2 *rhotar, const double2 *states, double *gpart,
                            hipStream_t st) {
  if (nitems == 0) return LB_OK;
#define X(B, E, C) \
  if (block == B && ept == E && Q == C) return adj_t<B, E, C>(p, d_items, nitems, kind, ctab, ktab, rhotar, states, gpart, st);
  LBX_FAST_SHAPES(X)
#undef X
  return fail(LB_EUNSUPPORTED, "no specialised LDS-resident kernel for this shape");
}

}  // namespace lbx
