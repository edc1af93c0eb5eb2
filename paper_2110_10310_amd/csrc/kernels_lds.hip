// LDS-resident persistent kernels for small systems (N^2 <= 4096).
//
// One workgroup owns one state of one system for the whole time loop: the
// stage iterate lives in two LDS buffers, the state q, the stage weights w
// and the digit tables of the thread's entries live in registers, and HBM is
// touched once per step only to store the state history that the adjoint
// pass reads.  The forward kernel runs every implicit-midpoint step of
// App. A; the adjoint kernel runs the discrete adjoint of App. B backwards
// and emits the per-step gradient integrands.
#include <hip/hip_runtime.h>

#include "lbx_host.hpp"

namespace lbx {

// A-priori sweep count of a step; a step whose contraction bound is >= 0.5
// (count -1) raises LB_STATUS_THETA and takes one sweep, so that the loop
// still ends.
__device__ __forceinline__ int a_priori_sweeps(int k, int32_t *status) {
  if (k >= 1) return k;
  if (status && threadIdx.x == 0) atomicOr(status, LB_STATUS_THETA);
  return 1;
}

template <int BLOCK, int EPT>
__global__ __launch_bounds__(BLOCK) void lds_forward_kernel(
    const SysDev *__restrict__ sysv, const LdsItem *__restrict__ items,
    const double *__restrict__ Etab, const uint64_t *__restrict__ desc,
    const double2 *__restrict__ ctab, const int32_t *__restrict__ ktab, int NT,
    const double2 *__restrict__ rho0, double2 *__restrict__ rhoT, double2 *__restrict__ states,
    int64_t *__restrict__ sweeps, int32_t *__restrict__ status) {
  extern __shared__ double2 zbuf[];  // two stage buffers of N^2 entries
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dsh[2][QMAX];
  __shared__ double2 jsh[2][JCMAX];
  const LdsItem it = items[blockIdx.x];
  const SysDev &S = sysv[it.sys];
  const int tid = threadIdx.x;
  const int N = S.N;
  const int64_t N2 = S.N2;
  const double h = S.h;
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);

  // Per entry: state q, stage weight w = (1 - h D)^-1 and h D.  The stage
  // vector is carried as z = q + delta and only delta is iterated:
  //   delta <- w (h D q + h O z),   q^{j+1} = q^j + 2 delta,
  // which solves the same system as z <- w (q + h O z) but never rounds
  // 1 + h*gamma (gamma ~ 1e-5/ns), whose rounding would repeat identically
  // every step and accumulate linearly.
  double2 qv[EPT], wv[EPT], hd[EPT], dn[EPT];
  uint64_t di[EPT], dj[EPT];
  int ee[EPT];
  bool ok[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * BLOCK;
    ok[k] = e < N2;
    ee[k] = ok[k] ? e : 0;
    const int i = ee[k] / N;
    const int jj = ee[k] - i * N;
    di[k] = desc[S.tab_off + i];
    dj[k] = desc[S.tab_off + jj];
    const double gam = diag_rate(S, di[k], dj[k]);
    const double dE = Etab[S.tab_off + i] - Etab[S.tab_off + jj];
    wv[k] = stage_weight(h, gam, dE, false);
    hd[k] = cscale(h, diag_coef(gam, dE, false));
    qv[k] = ok[k] ? rho0[it.off + e] : make_double2(0.0, 0.0);
    dn[k] = make_double2(0.0, 0.0);
    if (states && ok[k]) states[it.st_off + e] = qv[k];
  }
  // Two LDS stage buffers; selected by value (not through a pointer array)
  // so that every access stays an LDS instruction.
  double2 *const zb0 = zbuf, *const zb1 = zbuf + N2;
  int cb = 0;
  int64_t nsw = 0;
  for (int j = 0; j < NT; ++j) {
    // (I - h M) z = q^j (App. A eq. linsystem_primal): z0 = w q, then K sweeps.
    double2 hdq[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      hdq[k] = cmul(hd[k], qv[k]);
      if (ok[k]) (cb ? zb1 : zb0)[ee[k]] = cadd(qv[k], cmul(wv[k], hdq[k]));
    }
    if (tid < S.Q) dsh[j & 1][tid] = ctab[S.ctab_off + (int64_t)j * S.Q + tid];
    if (tid < S.njc) jsh[j & 1][tid] = jc_coef(S, tid, ((double)j + 0.5) * S.dt);
    __syncthreads();
    const int K = a_priori_sweeps(ktab[((int64_t)it.sys * NT + j) * 2 + 0], status);
    nsw += K;
    for (int kk = 0; kk < K; ++kk) {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        if (ok[k]) {
          const double2 acc = offdiag_all<false>(S, di[k], dj[k], ee[k], dsh[j & 1], jsh[j & 1], sq,
                                             [&](int64_t idx) { return src[idx]; });
          dn[k] = cmul(wv[k], cadd(hdq[k], cscale(h, acc)));
        }
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
    // q^{j+1} = q^j + dt M z = q^j + 2 delta (App. A eq. IMR; h M z = z - q^j = delta).
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      qv[k] = cadd(qv[k], cscale(2.0, dn[k]));
      if (states && ok[k]) states[it.st_off + (int64_t)(j + 1) * N2 + ee[k]] = qv[k];
    }
    cb ^= 1;
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k)
    if (ok[k]) rhoT[it.off + ee[k]] = qv[k];
  if (sweeps && tid == 0) sweeps[blockIdx.x] = nsw;
}

template <int BLOCK, int EPT>
__global__ __launch_bounds__(BLOCK) void lds_adjoint_kernel(
    const SysDev *__restrict__ sysv, const LdsItem *__restrict__ items,
    const double *__restrict__ Etab, const uint64_t *__restrict__ desc,
    const double2 *__restrict__ ctab, const int32_t *__restrict__ ktab, int NT, int kind,
    const double2 *__restrict__ rhotar, const double2 *__restrict__ states, const double *__restrict__ ptab,
    double *__restrict__ gpart, int64_t *__restrict__ sweeps, int32_t *__restrict__ status) {
  extern __shared__ double2 zbuf[];
  __shared__ double sq[SQRT_TABLE];
  __shared__ double2 dsh[2][QMAX];
  __shared__ double2 jsh[2][JCMAX];
  constexpr int WAVES = BLOCK / 64;
  const LdsItem it = items[blockIdx.x];
  const SysDev &S = sysv[it.sys];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int N = S.N;
  const int64_t N2 = S.N2;
  const double h = S.h;
  const int Q = S.Q;
  if (tid < SQRT_TABLE) sq[tid] = sqrt((double)tid);

  double2 qh[EPT], wv[EPT], hd[EPT], dn[EPT], qn[EPT], tg[EPT];
  uint64_t di[EPT], dj[EPT];
  int ee[EPT];
  bool ok[EPT];
  const double2 *hist = states + it.st_off;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = tid + k * BLOCK;
    ok[k] = e < N2;
    ee[k] = ok[k] ? e : 0;
    const int i = ee[k] / N;
    const int jj = ee[k] - i * N;
    di[k] = desc[S.tab_off + i];
    dj[k] = desc[S.tab_off + jj];
    const double gam = diag_rate(S, di[k], dj[k]);
    const double dE = Etab[S.tab_off + i] - Etab[S.tab_off + jj];
    wv[k] = stage_weight(h, gam, dE, true);
    hd[k] = cscale(h, diag_coef(gam, dE, true));
    // Terminal condition (App. B): qh = (beta/M) dJ/d(conj q) at q = rho(T).
    qn[k] = ok[k] ? hist[(int64_t)NT * N2 + ee[k]] : make_double2(0.0, 0.0);
    const double2 t = ok[k] ? rhotar[it.off + ee[k]] : make_double2(0.0, 0.0);
    tg[k] = t;
    qh[k] = kind == LB_J_FROB ? cscale(it.wterm, csub(qn[k], t)) : cscale(kind == LB_J_NM ? it.wterm : -it.wterm, t);
    dn[k] = make_double2(0.0, 0.0);
  }
  // Two LDS stage buffers; selected by value (not through a pointer array)
  // so that every access stays an LDS instruction.
  double2 *const zb0 = zbuf, *const zb1 = zbuf + N2;
  int cb = 0;
  int64_t nsw = 0;
  for (int j = NT - 1; j >= 0; --j) {
    // (I - h M^+) zh = qh^{j+1} (App. B eq. linsystem_adjoint), zh = qh + delta.
    double2 hdq[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      hdq[k] = cmul(hd[k], qh[k]);
      if (ok[k]) (cb ? zb1 : zb0)[ee[k]] = cadd(qh[k], cmul(wv[k], hdq[k]));
    }
    if (tid < Q) dsh[j & 1][tid] = ctab[S.ctab_off + (int64_t)j * Q + tid];
    if (tid < S.njc) jsh[j & 1][tid] = jc_coef(S, tid, ((double)j + 0.5) * S.dt);
    // Forward state q^j, consumed after the sweeps so that its load overlaps them.
    double2 qj[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) qj[k] = ok[k] ? hist[(int64_t)j * N2 + ee[k]] : make_double2(0.0, 0.0);
    __syncthreads();
    const int K = a_priori_sweeps(ktab[((int64_t)it.sys * NT + j) * 2 + 0], status);
    nsw += K;
    for (int kk = 0; kk < K; ++kk) {
      const double2 *src = (cb ? zb1 : zb0);
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        if (ok[k]) {
          const double2 acc = offdiag_all<true>(S, di[k], dj[k], ee[k], dsh[j & 1], jsh[j & 1], sq,
                                            [&](int64_t idx) { return src[idx]; });
          dn[k] = cmul(wv[k], cadd(hdq[k], cscale(h, acc)));
        }
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
    // Gradient integrands need zh = qh + delta at neighbours: publish it.
    double2 *zhb = (cb ? zb0 : zb1);
#pragma unroll
    for (int k = 0; k < EPT; ++k)
      if (ok[k]) zhb[ee[k]] = cadd(qh[k], dn[k]);
    __syncthreads();
    for (int q = 0; q < Q; ++q) {
      double gp = 0.0, gq = 0.0;
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        if (ok[k]) {
          const double2 z = cscale(0.5, cadd(qj[k], qn[k]));
          grad_term(S, q, di[k], dj[k], ee[k], z, sq, [&](int64_t idx) { return zhb[idx]; }, gp,
                    gq);
        }
      }
      gp = wave_sum<64>(gp);
      gq = wave_sum<64>(gq);
      if (lane == 0) {
        double *dstp = gpart + it.gp_off + ((int64_t)j * WAVES + wave) * 2 * Q + 2 * q;
        dstp[0] = gp;
        dstp[1] = gq;
      }
    }
    // qh^j = qh^{j+1} + dt M^+ zh = qh^{j+1} + 2 delta, plus the source of the
    // running penalty (App. B), w dJ/d(conj q^j) with w = gamma1 dt beta(t_j) / M
    // (it has no effect on the gradient at j = 0).
    const double wp = (ptab && j > 0) ? it.wpen * ptab[(int64_t)it.sys * NT + j] : 0.0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      qh[k] = cadd(qh[k], cscale(2.0, dn[k]));
      if (wp != 0.0)
        qh[k] = cadd(qh[k], cscale(wp, kind == LB_J_FROB ? csub(qj[k], tg[k])
                                                          : (kind == LB_J_NM ? tg[k] : cscale(-1.0, tg[k]))));
      qn[k] = qj[k];
    }
    // The next step writes its first iterate into (cb ? zb1 : zb0): the last sweep's
    // reads of it finished before the barrier above.
  }
  if (sweeps && tid == 0) sweeps[blockIdx.x] = nsw;
}

bool lds_shape(int64_t n2, int *block, int *ept) {
  if (n2 <= 64) { *block = 64; *ept = 1; }
  else if (n2 <= 128) { *block = 128; *ept = 1; }
  else if (n2 <= 256) { *block = 256; *ept = 1; }
  else if (n2 <= 512) { *block = 512; *ept = 1; }
  else if (n2 <= 1024) { *block = 1024; *ept = 1; }
  else if (n2 <= 2048) { *block = 1024; *ept = 2; }
  else if (n2 <= 4096) { *block = 1024; *ept = 4; }
  else return false;
  return true;
}

template <int BLOCK, int EPT>
static int launch_fwd_t(const lb_plan *p, const LdsItem *d_items, int nitems, size_t shmem,
                        const double2 *ctab, const int32_t *ktab, const double2 *rho0,
                        double2 *rhoT, double2 *states, int64_t *sweeps, int32_t *status, hipStream_t st) {
  auto kern = lds_forward_kernel<BLOCK, EPT>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shmem));
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(BLOCK), shmem, st, p->d_sys, d_items, p->d_E,
                     p->d_desc, ctab, ktab, p->NT, rho0, rhoT, states, sweeps, status);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

template <int BLOCK, int EPT>
static int launch_adj_t(const lb_plan *p, const LdsItem *d_items, int nitems, size_t shmem,
                        int kind, const double2 *ctab, const int32_t *ktab,
                        const double2 *rhotar, const double2 *states, const double *ptab, double *gpart,
                        int64_t *sweeps, int32_t *status, hipStream_t st) {
  auto kern = lds_adjoint_kernel<BLOCK, EPT>;
  LBX_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)shmem));
  hipLaunchKernelGGL(kern, dim3(nitems), dim3(BLOCK), shmem, st, p->d_sys, d_items, p->d_E,
                     p->d_desc, ctab, ktab, p->NT, kind, rhotar, states, ptab, gpart, sweeps, status);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

static size_t lds_bytes(int block, int ept) { return (size_t)2 * block * ept * sizeof(double2); }

int launch_lds_forward(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                       const double2 *ctab, const int32_t *ktab, const double2 *rho0,
                       double2 *rhoT, double2 *states, int64_t *sweeps, int32_t *status, hipStream_t st) {
  if (nitems == 0) return LB_OK;
  const size_t sh = lds_bytes(block, ept);
#define LBX_FWD(Bk, Ep) \
  if (block == Bk && ept == Ep) return launch_fwd_t<Bk, Ep>(p, d_items, nitems, sh, ctab, ktab, rho0, rhoT, states, sweeps, status, st);
  LBX_FWD(64, 1) LBX_FWD(128, 1) LBX_FWD(256, 1) LBX_FWD(512, 1) LBX_FWD(1024, 1)
  LBX_FWD(1024, 2) LBX_FWD(1024, 4)
#undef LBX_FWD
  return fail(LB_EUNSUPPORTED, "no LDS-resident kernel for this state size");
}

int launch_lds_adjoint(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                       int kind, const double2 *ctab, const int32_t *ktab, const double2 *rhotar,
                       const double2 *states, const double *ptab, double *gpart, int64_t *sweeps,
                       int32_t *status, hipStream_t st) {
  if (nitems == 0) return LB_OK;
  const size_t sh = lds_bytes(block, ept);
#define LBX_ADJ(Bk, Ep) \
  if (block == Bk && ept == Ep) return launch_adj_t<Bk, Ep>(p, d_items, nitems, sh, kind, ctab, ktab, rhotar, states, ptab, gpart, sweeps, status, st);
  LBX_ADJ(64, 1) LBX_ADJ(128, 1) LBX_ADJ(256, 1) LBX_ADJ(512, 1) LBX_ADJ(1024, 1)
  LBX_ADJ(1024, 2) LBX_ADJ(1024, 4)
#undef LBX_ADJ
  return fail(LB_EUNSUPPORTED, "no LDS-resident kernel for this state size");
}

// gstep[s][j][c] = sum over the items of s and their partial sums (fixed order).
__global__ void lds_grad_reduce_kernel(const SysDev *__restrict__ sysv,
                                       const int32_t *__restrict__ item_range,
                                       const int32_t *__restrict__ sys_ids,
                                       const LdsItem *__restrict__ items, int NT,
                                       const double *__restrict__ gpart,
                                       double *__restrict__ gstep) {
  const int ls = blockIdx.y;
  const int s = sys_ids[ls];
  const SysDev &S = sysv[s];
  const int twoQ = 2 * S.Q;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)NT * twoQ) return;
  const int j = (int)(idx / twoQ);
  const int c = (int)(idx - (int64_t)j * twoQ);
  double v = 0.0;
  for (int k = item_range[ls]; k < item_range[ls + 1]; ++k) {
    const LdsItem &it = items[k];
    const double *g = gpart + it.gp_off + (int64_t)j * it.parts * twoQ + c;
    for (int w = 0; w < it.parts; ++w) v += g[w * twoQ];
  }
  gstep[2 * S.ctab_off + idx] = v;
}

int launch_lds_grad_reduce(const lb_plan *p, const int32_t *d_item_range, int nsys_lds,
                           const int32_t *d_sys_ids, const LdsItem *d_items, const double *gpart,
                           double *gstep, hipStream_t st) {
  if (nsys_lds == 0) return LB_OK;
  int qmax = 1;
  for (const auto &s : p->sys) qmax = s.Q > qmax ? s.Q : qmax;
  const int64_t n = (int64_t)p->NT * 2 * qmax;
  hipLaunchKernelGGL(lds_grad_reduce_kernel, dim3((unsigned)((n + 255) / 256), nsys_lds), dim3(256),
                     0, st, p->d_sys, d_item_range, d_sys_ids, d_items, p->NT, gpart, gstep);
  LBX_HIP(hipGetLastError());
  return LB_OK;
}

}  // namespace lbx
