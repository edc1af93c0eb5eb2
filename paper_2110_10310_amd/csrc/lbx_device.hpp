// Device-side data structures and the matrix-free Lindbladian stencil.
//
// Notation (paper Sec. II, App. A): an entry (i, j) of a density matrix has
// row digits n_q (levels of basis index i) and column digits m_q (levels of
// j), subsystem 0 most significant.  M = D + O where
//   D_ij = -i (E_i - E_j) - gamma_ij,
//   gamma_ij = sum_q [ (n_q + m_q) / (2 T1_q) + (n_q - m_q)^2 / (2 T2_q) ]
// holds H_sys (diagonal: detuning, self- and cross-Kerr), the dephasing
// dissipator and the decay anticommutator, and O holds the control
// commutator -i[H_c, .] (ladder shifts of one row or one column digit) and
// the decay jump a rho a^+ / T1 (shift of both digits of one subsystem).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbx.h"

namespace lbx {

constexpr int QMAX = LB_LIMIT_QMAX;
constexpr int DIGIT_BITS = 5;
constexpr int SQRT_TABLE = 33;  // sqrt(k) for k = 0..32
constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr int JCMAX = QMAX * (QMAX - 1) / 2;  // Jaynes-Cummings pairs p > q

// Per-system constants.  One array of these lives in device memory per plan.
struct SysDev {
  int32_t Q, N, NT, Ns, Nf, nalpha;
  int64_t N2;
  int32_t nlev[QMAX];
  int32_t stride[QMAX];  // basis-index stride of subsystem q
  double g1[QMAX];       // 1/T1_q, 0 when off
  double g2[QMAX];       // 1/T2_q, 0 when off
  double csum[QMAX];     // max over n of sqrt(n)[n>0] + sqrt(n+1)[n+1<nlev]
  double T, dt, h;       // h = dt/2
  double dtau;           // B-spline knot spacing T/(Ns-2)
  double theta_jump;     // h * sum_q (nlev_q - 1)/T1_q, plus the coupling bound
  double hDmax;          // h * max_ij |D_ij|
  int64_t tab_off;       // first row of this system in the energy/digit tables
  int64_t carrier_off;   // first entry in the carrier table ([Q][Nf])
  int64_t alpha_off;     // first entry in a concatenated alpha
  int64_t ctab_off;      // first entry in the control table ([NT][Q] complex)
  // Jaynes-Cummings coupling (Sec. II): pair k couples subsystems jp[k] > jq[k]
  // with g = jg[k] (rad/ns) and phase rate jd[k] = w_p^rot - w_q^rot (rad/ns).
  int32_t njc;
  int8_t jp[JCMAX], jq[JCMAX];
  double jg[JCMAX], jd[JCMAX];
};

__device__ __forceinline__ int digit(uint64_t packed, int q) {
  return (int)((packed >> (DIGIT_BITS * q)) & ((1u << DIGIT_BITS) - 1));
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// gamma_ij: decay anticommutator plus dephasing, both real and diagonal.
__device__ __forceinline__ double diag_rate(const SysDev &S, uint64_t di, uint64_t dj) {
  double g = 0.0;
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    if (q < S.Q) {
      const int n = digit(di, q), m = digit(dj, q);
      const double dnm = (double)(n - m);
      g += 0.5 * (S.g1[q] * (double)(n + m) + S.g2[q] * dnm * dnm);
    }
  }
  return g;
}

// D_ij (forward) or conj(D_ij) (adjoint).
__device__ __forceinline__ double2 diag_coef(double gam, double dE, bool adj) {
  return make_double2(-gam, adj ? dE : -dE);
}

// w_ij = 1 / (1 - h D_ij) (forward) or its conjugate (adjoint).
// 1 - h D_ij = (1 + h gamma_ij) + i h (E_i - E_j).
__device__ __forceinline__ double2 stage_weight(double h, double gam, double dE, bool adj) {
  const double re = 1.0 + h * gam;
  const double im = h * dE;
  const double inv = 1.0 / (re * re + im * im);
  return make_double2(re * inv, adj ? im * inv : -im * inv);
}

// The off-diagonal part O x at flat entry r = i*N + j of one state (forward)
// or O^+ x (adjoint).  `ld(idx)` returns x at flat entry idx of the same
// state; it is only called with in-range indices.  dq[q] = d_q(t) in rad/ns.
//
// Control commutator, forward:
//   -i [ d sqrt(n+1) x_{i+e,j} + d* sqrt(n) x_{i-e,j}
//        - d sqrt(m) x_{i,j-e} - d* sqrt(m+1) x_{i,j+e} ]
//   = -i (d U + d* V),  U = sqrt(n+1) x_{i+e,j} - sqrt(m) x_{i,j-e},
//                        V = sqrt(n) x_{i-e,j} - sqrt(m+1) x_{i,j+e};
// the adjoint (+i [H_c, .]) flips the sign.  Decay jump, forward:
// sqrt((n+1)(m+1))/T1 x_{i+e,j+e}; adjoint: sqrt(n m)/T1 x_{i-e,j-e}.
// offdiag_range: the terms of subsystems q0 <= q < q1 only (the off-diagonal
// part is a sum over subsystems, so disjoint ranges add up to offdiag).
template <bool ADJ, class Load>
__device__ __forceinline__ double2 offdiag_range(const SysDev &S, uint64_t di, uint64_t dj, int64_t r,
                                                 const double2 *dq, const double *sq, Load ld, int q0, int q1) {
  double2 acc = make_double2(0.0, 0.0);
  const int64_t N = S.N;
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    if (q >= q0 && q < q1) {
      const int n = digit(di, q), m = digit(dj, q);
      const int nl = S.nlev[q];
      const int64_t s1 = S.stride[q];
      const int64_t sN = s1 * N;
      const bool rp = n + 1 < nl, rm = n > 0, cp = m + 1 < nl, cm = m > 0;
      const double2 xrp = ld(rp ? r + sN : r);
      const double2 xrm = ld(rm ? r - sN : r);
      const double2 xcp = ld(cp ? r + s1 : r);
      const double2 xcm = ld(cm ? r - s1 : r);
      const double arp = rp ? sq[n + 1] : 0.0;
      const double arm = sq[n];
      const double acp = cp ? sq[m + 1] : 0.0;
      const double acm = sq[m];
      const double2 U = csub(cscale(arp, xrp), cscale(acm, xcm));
      const double2 V = csub(cscale(arm, xrm), cscale(acp, xcp));
      const double2 Sm = cadd(U, V);
      const double2 Dv = csub(U, V);
      const double a = dq[q].x, b = dq[q].y;
      double2 ctl = make_double2(a * Sm.y + b * Dv.x, -a * Sm.x + b * Dv.y);
      if (ADJ) ctl = make_double2(-ctl.x, -ctl.y);
      double2 jmp;
      if (!ADJ) {
        const bool ok = rp && cp;
        const double c = ok ? S.g1[q] * sq[n + 1] * sq[m + 1] : 0.0;
        jmp = cscale(c, ld(ok ? r + sN + s1 : r));
      } else {
        const bool ok = rm && cm;
        const double c = ok ? S.g1[q] * sq[n] * sq[m] : 0.0;
        jmp = cscale(c, ld(ok ? r - sN - s1 : r));
      }
      acc = cadd(acc, cadd(ctl, jmp));
    }
  }
  return acc;
}

template <bool ADJ, class Load>
__device__ __forceinline__ double2 offdiag(const SysDev &S, uint64_t di, uint64_t dj, int64_t r,
                                           const double2 *dq, const double *sq, Load ld) {
  return offdiag_range<ADJ>(S, di, dj, r, dq, sq, ld, 0, S.Q);
}

// Coefficient c_k = g e^{i Delta t} of Jaynes-Cummings pair k at time t.
__device__ __forceinline__ double2 jc_coef(const SysDev &S, int k, double t) {
  double sn, cs;
  sincos(S.jd[k] * t, &sn, &cs);
  return make_double2(S.jg[k] * cs, S.jg[k] * sn);
}

// The Jaynes-Cummings part of O x at entry r = i*N + j (Sec. II coupling
// sum_{p>q} c a_p^+ a_q + c* a_p a_q^+, c = jq[k]; forward: -i [H, x]):
//   -i [ c sqrt(n_p) sqrt(n_q+1) x_{i-e_p+e_q, j} + c* sqrt(n_p+1) sqrt(n_q) x_{i+e_p-e_q, j}
//        - c sqrt(m_p+1) sqrt(m_q) x_{i, j+e_p-e_q} - c* sqrt(m_p) sqrt(m_q+1) x_{i, j-e_p+e_q} ]
// (n, m: digits of i, j); the adjoint (+i [H, x]) flips the sign.
template <bool ADJ, class Load>
__device__ __forceinline__ double2 jc_terms(const SysDev &S, uint64_t di, uint64_t dj, int64_t r,
                                            const double2 *jq, const double *sq, Load ld) {
  double2 acc = make_double2(0.0, 0.0);
  const int64_t N = S.N;
  for (int k = 0; k < S.njc; ++k) {
    const int p = S.jp[k], q = S.jq[k];
    const int np = digit(di, p), nq = digit(di, q), mp = digit(dj, p), mq = digit(dj, q);
    const int lp = S.nlev[p], lq = S.nlev[q];
    const int64_t sp = S.stride[p], sqs = S.stride[q];
    const double2 c = jq[k];
    const double2 cc = make_double2(c.x, -c.y);
    // row part
    const bool r1 = np > 0 && nq + 1 < lq, r2 = np + 1 < lp && nq > 0;
    const double w1 = r1 ? sq[np] * sq[nq + 1] : 0.0, w2 = r2 ? sq[np + 1] * sq[nq] : 0.0;
    const double2 x1 = ld(r1 ? r + (sqs - sp) * N : r), x2 = ld(r2 ? r + (sp - sqs) * N : r);
    // column part
    const bool c1 = mp + 1 < lp && mq > 0, c2 = mp > 0 && mq + 1 < lq;
    const double v1 = c1 ? sq[mp + 1] * sq[mq] : 0.0, v2 = c2 ? sq[mp] * sq[mq + 1] : 0.0;
    const double2 y1 = ld(c1 ? r + (sp - sqs) : r), y2 = ld(c2 ? r + (sqs - sp) : r);
    const double2 u = csub(cadd(cscale(w1, cmul(c, x1)), cscale(w2, cmul(cc, x2))),
                           cadd(cscale(v1, cmul(c, y1)), cscale(v2, cmul(cc, y2))));
    // -i u (forward), +i u (adjoint)
    acc = ADJ ? cadd(acc, make_double2(-u.y, u.x)) : cadd(acc, make_double2(u.y, -u.x));
  }
  return acc;
}

// offdiag plus the coupling (jq may be NULL when the system has none).
template <bool ADJ, class Load>
__device__ __forceinline__ double2 offdiag_all(const SysDev &S, uint64_t di, uint64_t dj, int64_t r,
                                               const double2 *dq, const double2 *jq, const double *sq, Load ld) {
  double2 acc = offdiag<ADJ>(S, di, dj, r, dq, sq, ld);
  if (S.njc > 0) acc = cadd(acc, jc_terms<ADJ>(S, di, dj, r, jq, sq, ld));
  return acc;
}

// Gradient integrands of one entry for subsystem q (App. B eq.
// reducedgradient through p_q = Re d_q and q_q = Im d_q):
//   gp += Re <zh, X_q z>, X_q = -i[a_q + a_q^+, .] = dM/dp_q,
//   gq += Re <zh, Y_q z>, Y_q = [a_q - a_q^+, .] = dM/dq_q,
// evaluated as -Re <X_q zh, z> and -Re <Y_q zh, z> (X_q and Y_q are
// skew-adjoint), so only zh needs neighbours: with U, V as in `offdiag`
// built on zh, X_q zh = -i (U + V) and Y_q zh = U - V.
template <class Load>
__device__ __forceinline__ void grad_term(const SysDev &S, int q, uint64_t di, uint64_t dj,
                                          int64_t r, double2 z, const double *sq, Load ldzh,
                                          double &gp, double &gq) {
  const int64_t N = S.N;
  const int n = digit(di, q), m = digit(dj, q);
  const int nl = S.nlev[q];
  const int64_t s1 = S.stride[q];
  const int64_t sN = s1 * N;
  const bool rp = n + 1 < nl, rm = n > 0, cp = m + 1 < nl, cm = m > 0;
  const double2 xrp = ldzh(rp ? r + sN : r);
  const double2 xrm = ldzh(rm ? r - sN : r);
  const double2 xcp = ldzh(cp ? r + s1 : r);
  const double2 xcm = ldzh(cm ? r - s1 : r);
  const double2 U = csub(cscale(rp ? sq[n + 1] : 0.0, xrp), cscale(sq[m], xcm));
  const double2 V = csub(cscale(sq[n], xrm), cscale(cp ? sq[m + 1] : 0.0, xcp));
  const double2 Sm = cadd(U, V);
  const double2 Dv = csub(U, V);
  gp += Sm.x * z.y - Sm.y * z.x;
  gq -= Dv.x * z.x + Dv.y * z.y;
}

// Quadratic B-spline basis S_s(t) = B(t/dtau - s + 1/2), B the centred
// quadratic B-spline (Sec. II, knot spacing dtau, centres (s - 1/2) dtau).
__device__ __forceinline__ double bspline2(double x) {
  const double ax = fabs(x);
  if (ax <= 0.5) return 0.75 - ax * ax;
  if (ax <= 1.5) {
    const double u = ax - 1.5;
    return 0.5 * u * u;
  }
  return 0.0;
}

// d_q(t) of eq. (rotctrl) in rad/ns; alpha points at this system's [Q][Ns][Nf][2].
// Only splines whose support holds t contribute (at most three, found from
// t / dtau with one spline of margin on each side); each carrier's phase
// factor multiplies the spline sum of its coefficients.
__device__ inline double2 control_value(const SysDev &S, const double *alpha, const double *carrier,
                                        int q, double t) {
  const double u = t / S.dtau;
  const int fu = (int)floor(u);
  const int s0 = max(fu - 1, 0), s1 = min(fu + 3, S.Ns - 1);
  double re = 0.0, im = 0.0;
  for (int f = 0; f < S.Nf; ++f) {
    double ar = 0.0, ai = 0.0;
    for (int s = s0; s <= s1; ++s) {
      const double B = bspline2(u - (double)s + 0.5);
      ar += B * alpha[((q * S.Ns + s) * S.Nf + f) * 2 + 0];
      ai += B * alpha[((q * S.Ns + s) * S.Nf + f) * 2 + 1];
    }
    double sn, cs;
    sincos(TWO_PI * carrier[q * S.Nf + f] * t, &sn, &cs);
    re += ar * cs - ai * sn;
    im += ar * sn + ai * cs;
  }
  return make_double2(TWO_PI * re, TWO_PI * im);
}

template <int W>
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

}  // namespace lbx
