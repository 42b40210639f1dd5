// hrm_device.hpp -- gfx950 device arithmetic of the hot path: mixture EOS,
// characteristic projection, incremental-stencil WENO, HLLC, HCS
// reconstruction with shock-sensor blending, the positivity-preserving
// interpolation and flux limiters, and the infinite-rate thermal relaxation
// (Wong, Angel & Kiris, arXiv:2208.04488, Sec. 2, Sec. 4, App. C, App. D).
//
// Face arithmetic is templated on R (double, or float for the FP32 variant);
// the node primitives, the flux limiter, every limiter bound check, the
// accumulation and the relaxation are double in both.  Component slots of a
// conservative vector W (Sec. 2): alpha_k rho_k (k < N), rho u_d (d < D), E,
// alpha_k (k < N-1).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace hrm {

constexpr int MAXN = 8;

// grid flags (mirror of the public header)
constexpr int F_NO_LIMITERS = 1;
constexpr int F_NO_BLEND = 2;
constexpr int F_FIRST_ORDER = 4;
constexpr int F_FOUR_EQ = 32;  // the four-equation HRM solved directly (first-order HLLC)

// species table with the derived constants every kernel needs
struct EosDev {
    double g[MAXN], cv[MAXN], pinf[MAXN], q[MAXN];
    double ig1[MAXN];   // 1/(gamma_k - 1)
    double gpi1[MAXN];  // gamma_k pinf_k/(gamma_k - 1)
    double cp[MAXN];    // gamma_k c_v,k
};

struct MlpPacked;  // learned interpolation weights (hrm_mlp.hpp)

struct ParDev {
    double eps_weno;
    double eps_i_ar, eps_i_a, hs_i_ar, hs_i_a, hs_i_rc2;
    double eps_f_ar, eps_f_a, eps_f_re, hs_f_ar, hs_f_a, hs_f_re;
    double Cs, qexp, psi;
    double hcs_a, hcs_b, hcs_c;  // eq:reconstructed_G coefficients from psi
    int flags;
    int fast_flux_limiter;  // eps_f >= eps_f^HS for all three quantities
    const MlpPacked* mlp;   // packed network of the learned weights (device), or null
};

// counters accumulated per thread, flushed once per wave
enum { C_ALG1 = 0, C_ALG2, C_IHS, C_ALG3, C_ALG4, C_FHS, C_RELAX_BAD, C_N };

// The counts of one face (and one cell update) packed into one register, 4
// bits per counter: a face blends at most 2N <= 6 partial densities (Alg. 1)
// and 2 volume-fraction sets (Alg. 2), switches at most twice, limits its
// flux once.  One register instead of seven live through the face.
constexpr unsigned cnt_one(int k) { return 1u << (4 * k); }
__device__ inline unsigned cnt_get(unsigned packed, int k) { return (packed >> (4 * k)) & 15u; }

// A full state: conservative and primitive slots side by side.
template <int N, int D, typename R = double>
struct St {
    R ar[N];   // alpha_k rho_k
    R mom[D];  // rho u_d
    R u[D];
    R p, E;
    double al[N];  // all N volume fractions, al[N-1] = 1 - sum of the others (always double:
                   // a bulk fraction 1 - 1e-8 next to a trace 1e-8 is not representable in float)
    R rho, c, rc2;
};

// a state converted to another arithmetic type
template <int N, int D, typename R, typename S>
__device__ inline St<N, D, R> convert(const St<N, D, S>& s)
{
    St<N, D, R> o;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        o.ar[k] = (R)s.ar[k];
        o.al[k] = s.al[k];
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        o.mom[d] = (R)s.mom[d];
        o.u[d] = (R)s.u[d];
    }
    o.p = (R)s.p;
    o.E = (R)s.E;
    o.rho = (R)s.rho;
    o.c = (R)s.c;
    o.rc2 = (R)s.rc2;
    return o;
}

// Sec. 2 mixture EOS: Gam = 1/(gbar-1) = sum alpha_k/(gamma_k-1),
// Pi = gbar pbar/(gbar-1) = sum alpha_k gamma_k pinf_k/(gamma_k-1);
// rho(e - qbar) = Gam p + Pi; rho c^2 = gbar (p + pbar) = p + (p + Pi)/Gam.
template <int N, typename R>
__device__ inline void mixture(const EosDev& e, const R* al, R& Gam, R& Pi)
{
    Gam = 0;
    Pi = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        Gam += al[k] * (R)e.ig1[k];
        Pi += al[k] * (R)e.gpi1[k];
    }
}

// 1/x from the hardware reciprocal refined by two Newton steps: within about
// an ulp of the IEEE quotient, in 5 instructions instead of the ~10 of an
// IEEE division.  x must be a normal number (not 0, infinite, NaN or
// subnormal), as the WENO-IS weight sums and the densities and mixture
// Gamma of cells are; elsewhere the IEEE quotient is kept.
__device__ inline double rcp_newton(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}

// conservative W[M] -> full state (hot-path step a1)
template <int N, int D>
__device__ inline void state_from_W(const EosDev& e, const double* W, St<N, D>& s)
{
    constexpr int IE = N + D, IA = N + D + 1;
    double rho = 0.0, rq = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        s.ar[k] = W[k];
        rho += W[k];
        rq += W[k] * e.q[k];
    }
    double asum = 0.0;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        s.al[k] = W[IA + k];
        asum += W[IA + k];
    }
    s.al[N - 1] = 1.0 - asum;
    const double irho = rcp_newton(rho);
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        s.mom[d] = W[N + d];
        s.u[d] = W[N + d] * irho;
        m2 += W[N + d] * W[N + d];
    }
    double Gam, Pi;
    mixture<N>(e, s.al, Gam, Pi);
    const double iG = rcp_newton(Gam);
    s.E = W[IE];
    const double re = W[IE] - 0.5 * m2 * irho - rq;
    s.p = (re - Pi) * iG;
    s.rc2 = s.p + (s.p + Pi) * iG;
    s.rho = rho;
    s.c = sqrt(s.rc2 * irho);
}

// primitive slots (ar, u, p, al[0..N-2]) already set -> the rest of the state
template <int N, int D, typename R>
__device__ inline void complete_from_prim(const EosDev& e, St<N, D, R>& s)
{
    R rho = 0, rq = 0;
    double asum = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        rho += s.ar[k];
        rq += s.ar[k] * (R)e.q[k];
    }
#pragma unroll
    for (int k = 0; k < N - 1; ++k) asum += s.al[k];
    s.al[N - 1] = 1.0 - asum;
    double Gd, Pd;
    mixture<N, double>(e, s.al, Gd, Pd);
    const R Gam = (R)Gd, Pi = (R)Pd;
    R u2 = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        s.mom[d] = rho * s.u[d];
        u2 += s.u[d] * s.u[d];
    }
    s.rho = rho;
    s.E = Gam * s.p + Pi + (R)0.5 * rho * u2 + rq;
    s.rc2 = s.p + (s.p + Pi) / Gam;
    s.c = sqrt(s.rc2 / rho);
}

// rho(e - qbar) of a conservative vector
template <int N, int D>
__device__ inline double rhoe_tilde(const EosDev& e, const double* W)
{
    double rho = 0.0, rq = 0.0, m2 = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        rho += W[k];
        rq += W[k] * e.q[k];
    }
#pragma unroll
    for (int d = 0; d < D; ++d) m2 += W[N + d] * W[N + d];
    return W[N + D] - 0.5 * m2 / rho - rq;
}

// App. C incremental-stencil WENO, left-biased at i+1/2 from u_{i-2..i+2}.
// The four unnormalised weights are scaled by the common product of the
// denominators so the weighting needs one reciprocal instead of six divisions.  The
// product spans up to ~1e-75..1e55 for the ranges met here, which double
// holds; in the FP32 variant the candidates and smoothness indicators are
// float and only this weighting is done in double.
template <typename R>
__device__ inline R weno_is_weigh(R s0, R s1, R s2, R s3, R q0, R q1, R q01, R q2, R q3, R qt, double eps)
{
    // weights (double): eta_k times Q = B0 B1 B01 B2 B3, B = beta + eps
    const double B0 = (double)q0 + eps, B1 = (double)q1 + eps, B01 = (double)q01 + eps;
    const double B2 = (double)q2 + eps, B3 = (double)q3 + eps, tau = qt;
    const double t2 = tau * tau;
    const double B23 = B2 * B3, B0B1 = B0 * B1;
    const double e0 = (15.0 / 32.0) * (B0 * B01 + t2) * B1 * B23;
    const double e1 = (5.0 / 32.0) * (B1 * B01 + t2) * B0 * B23;
    const double e2 = (5.0 / 16.0) * (B2 + tau) * B0B1 * B01 * B3;
    const double e3 = (1.0 / 16.0) * (B3 + tau) * B0B1 * B01 * B2;
    if constexpr (sizeof(R) == sizeof(double)) {
        return (e0 * s0 + e1 * s1 + e2 * s2 + e3 * s3) * rcp_newton(e0 + e1 + e2 + e3);
    } else {
        const double inv = rcp_newton(e0 + e1 + e2 + e3);
        return (R)(e0 * inv) * s0 + (R)(e1 * inv) * s1 + (R)(e2 * inv) * s2 + (R)(e3 * inv) * s3;
    }
}

template <typename R>
__device__ inline R weno_is(R um2, R um1, R u0, R up1, R up2, double eps)
{
    const R s0 = (R)0.5 * (u0 + up1);
    const R s1 = (R)0.5 * ((R)3 * u0 - um1);
    const R s2 = (R)0.125 * ((R)3 * u0 + (R)6 * up1 - up2);
    const R s3 = (R)0.125 * ((R)3 * um2 - (R)10 * um1 + (R)15 * u0);
    const R a0 = u0 - up1, a1 = um1 - u0;
    const R b01a = um1 - (R)2 * u0 + up1, b01b = um1 - up1;
    const R b2a = u0 - (R)2 * up1 + up2, b2b = (R)3 * u0 - (R)4 * up1 + up2;
    const R b3a = um2 - (R)2 * um1 + u0, b3b = um2 - (R)4 * um1 + (R)3 * u0;
    const R t5a = up2 - (R)4 * up1 + (R)6 * u0 - (R)4 * um1 + um2;
    const R t5b = up2 - (R)2 * up1 + (R)2 * um1 - um2;
    constexpr R c13 = (R)(13.0 / 12.0);
    const R q0 = a0 * a0, q1 = a1 * a1;
    const R q01 = c13 * b01a * b01a + (R)0.25 * b01b * b01b;
    const R q2 = c13 * b2a * b2a + (R)0.25 * b2b * b2b;
    const R q3 = c13 * b3a * b3a + (R)0.25 * b3b * b3b;
    const R qt = c13 * t5a * t5a + (R)0.25 * t5b * t5b;
    return weno_is_weigh<R>(s0, s1, s2, s3, q0, q1, q01, q2, q3, qt, eps);
}

// Both biased values at i+1/2 from v[0..5] = u_{i-2..i+3}: the left-biased
// weno_is(v0..v4) and the right-biased weno_is of the mirrored stencil
// v5..v1.  The two share the candidate (u_i + u_{i+1})/2, beta_0 and the
// squared second differences about i and i+1 (beta_01 of one side has the
// second-difference term of beta_2 of the other), which are formed once.
template <typename R>
__device__ inline void weno_is_pair(const R* v, double eps, R& l, R& r)
{
    constexpr R c13 = (R)(13.0 / 12.0);
    const R s0 = (R)0.5 * (v[2] + v[3]);
    const R a0 = v[2] - v[3];
    const R q0 = a0 * a0;
    const R dA = v[1] - (R)2 * v[2] + v[3];  // second difference about i
    const R dB = v[2] - (R)2 * v[3] + v[4];  // second difference about i+1
    const R cA = c13 * dA * dA, cB = c13 * dB * dB;
    {
        const R s1 = (R)0.5 * ((R)3 * v[2] - v[1]);
        const R s2 = (R)0.125 * ((R)3 * v[2] + (R)6 * v[3] - v[4]);
        const R s3 = (R)0.125 * ((R)3 * v[0] - (R)10 * v[1] + (R)15 * v[2]);
        const R a1 = v[1] - v[2], b01b = v[1] - v[3], b2b = (R)3 * v[2] - (R)4 * v[3] + v[4];
        const R b3a = v[0] - (R)2 * v[1] + v[2], b3b = v[0] - (R)4 * v[1] + (R)3 * v[2];
        const R t5a = v[4] - (R)4 * v[3] + (R)6 * v[2] - (R)4 * v[1] + v[0];
        const R t5b = v[4] - (R)2 * v[3] + (R)2 * v[1] - v[0];
        const R q1 = a1 * a1;
        const R q01 = cA + (R)0.25 * b01b * b01b;
        const R q2 = cB + (R)0.25 * b2b * b2b;
        const R q3 = c13 * b3a * b3a + (R)0.25 * b3b * b3b;
        const R qt = c13 * t5a * t5a + (R)0.25 * t5b * t5b;
        l = weno_is_weigh<R>(s0, s1, s2, s3, q0, q1, q01, q2, q3, qt, eps);
    }
    {
        const R s1 = (R)0.5 * ((R)3 * v[3] - v[4]);
        const R s2 = (R)0.125 * ((R)3 * v[3] + (R)6 * v[2] - v[1]);
        const R s3 = (R)0.125 * ((R)3 * v[5] - (R)10 * v[4] + (R)15 * v[3]);
        const R a1 = v[4] - v[3], b01b = v[4] - v[2], b2b = (R)3 * v[3] - (R)4 * v[2] + v[1];
        const R b3a = v[5] - (R)2 * v[4] + v[3], b3b = v[5] - (R)4 * v[4] + (R)3 * v[3];
        const R t5a = v[1] - (R)4 * v[2] + (R)6 * v[3] - (R)4 * v[4] + v[5];
        const R t5b = v[1] - (R)2 * v[2] + (R)2 * v[4] - v[5];
        const R q1 = a1 * a1;
        const R q01 = cB + (R)0.25 * b01b * b01b;
        const R q2 = cA + (R)0.25 * b2b * b2b;
        const R q3 = c13 * b3a * b3a + (R)0.25 * b3b * b3b;
        const R qt = c13 * t5a * t5a + (R)0.25 * t5b * t5b;
        r = weno_is_weigh<R>(s0, s1, s2, s3, q0, q1, q01, q2, q3, qt, eps);
    }
}

// Sec. 4.1.1 HLLC for the five-equation model in direction DIR.  Writes
// G = F^HLLC + (0, ..., f_alpha) and returns s_*.  sign(0) = 0.
template <int N, int D, int DIR, typename R>
__device__ inline R hllc(const St<N, D, R>& L, const St<N, D, R>& Rs, double* G)
{
    constexpr int IE = N + D, IA = N + D + 1;
    const R uL = L.u[DIR], uR = Rs.u[DIR];
    const R ub = (R)0.5 * (uL + uR), cb = (R)0.5 * (L.c + Rs.c);
    const R sL = fmin(ub - cb, uL - L.c);
    const R sR = fmax(ub + cb, uR + Rs.c);
    const R dL = sL - uL, dR = sR - uR;
    const R ss = (Rs.p - L.p + L.rho * uL * dL - Rs.rho * uR * dR) / (L.rho * dL - Rs.rho * dR);
    const R sg = ss > (R)0 ? (R)1 : (ss < (R)0 ? (R)-1 : (R)0);
    const R wl = (R)0.5 * ((R)1 + sg), wr = (R)0.5 * ((R)1 - sg);
    const R sm = fmin((R)0, sL), sp = fmax((R)0, sR);
    if constexpr (sizeof(R) == sizeof(double)) {
        // star states U*_K = chi_K (...) with chi_K = (s_K - u_K) / (s_K - s*)
        const R chiL = dL / (sL - ss), chiR = dR / (sR - ss);
#pragma unroll
        for (int k = 0; k < N; ++k)
            G[k] = wl * (L.ar[k] * uL + sm * (chiL * L.ar[k] - L.ar[k])) +
                   wr * (Rs.ar[k] * uR + sp * (chiR * Rs.ar[k] - Rs.ar[k]));
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const R FLd = L.mom[d] * uL + (d == DIR ? L.p : (R)0);
            const R FRd = Rs.mom[d] * uR + (d == DIR ? Rs.p : (R)0);
            const R WsL = d == DIR ? chiL * L.rho * ss : chiL * L.rho * L.u[d];
            const R WsR = d == DIR ? chiR * Rs.rho * ss : chiR * Rs.rho * Rs.u[d];
            G[N + d] = wl * (FLd + sm * (WsL - L.mom[d])) + wr * (FRd + sp * (WsR - Rs.mom[d]));
        }
        const R EsL = chiL * (L.E + (ss - uL) * (L.rho * ss + L.p / dL));
        const R EsR = chiR * (Rs.E + (ss - uR) * (Rs.rho * ss + Rs.p / dR));
        G[IE] = wl * ((L.E + L.p) * uL + sm * (EsL - L.E)) + wr * ((Rs.E + Rs.p) * uR + sp * (EsR - Rs.E));
    } else {
        // float: the jumps U*_K - U_K in closed form.  chi_K - 1 =
        // (s* - u_K) / (s_K - s*) is far below float resolution when |s_K|
        // (a liquid's sound speed) dwarfs |s* - u_K|; chi_K U_K - U_K would
        // then round to 0 and drop the star-state correction of the flux.
        const R qL = (ss - uL) / (sL - ss), qR = (ss - uR) / (sR - ss);
#pragma unroll
        for (int k = 0; k < N; ++k)
            G[k] = wl * (L.ar[k] * uL + sm * (qL * L.ar[k])) + wr * (Rs.ar[k] * uR + sp * (qR * Rs.ar[k]));
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const R FLd = L.mom[d] * uL + (d == DIR ? L.p : (R)0);
            const R FRd = Rs.mom[d] * uR + (d == DIR ? Rs.p : (R)0);
            // chi (rho s*) - rho u = rho s_K q_K along DIR; chi m_d - m_d = q_K m_d across
            const R JL = d == DIR ? L.rho * sL * qL : qL * L.mom[d];
            const R JR = d == DIR ? Rs.rho * sR * qR : qR * Rs.mom[d];
            G[N + d] = wl * (FLd + sm * JL) + wr * (FRd + sp * JR);
        }
        // E*_K - E_K = q_K (E_K + p_K + rho_K s* (s_K - u_K))
        const R JL = qL * (L.E + L.p + L.rho * ss * dL);
        const R JR = qR * (Rs.E + Rs.p + Rs.rho * ss * dR);
        G[IE] = wl * ((L.E + L.p) * uL + sm * JL) + wr * ((Rs.E + Rs.p) * uR + sp * JR);
    }
#pragma unroll
    for (int k = 0; k < N - 1; ++k)
        G[IA + k] = (double)wl * (L.al[k] * (double)ss) + (double)wr * (Rs.al[k] * (double)ss);
    return ss;
}

// theta solving (1-theta) a + theta b = min(eps, a) when b < min(eps, a); else 1
__device__ inline double lim_theta(double a, double b, double eps)
{
    const double m = fmin(eps, a);
    return b < m ? (a - m) / (a - b) : 1.0;
}

// Sec. 4.3.2 interpolation limiter on an interpolated primitive state V
// (partial densities and volume fractions are blended toward the node state;
// velocity and pressure are kept), then the hard switch to the node state.
// On return V is a complete state (conservative slots, rho, c, rho c^2).
template <int N, int D, typename R>
__device__ inline void interp_limit(const EosDev& e, const ParDev& P, St<N, D, R>& V, const St<N, D, R>& node,
                                    unsigned& cnt)
{
#pragma unroll
    for (int k = 0; k < N; ++k) {  // Alg. 1
        const double a = node.ar[k], b = V.ar[k];
        const double m = fmin(P.eps_i_ar, a);
        if (b < m) {
            const double th = (a - m) / (a - b);
            V.ar[k] = (R)((1.0 - th) * a + th * b);
            cnt += cnt_one(C_ALG1);
        }
    }
    double at[N], asum = 0.0;  // Alg. 2
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        at[k] = V.al[k];
        asum += at[k];
    }
    at[N - 1] = 1.0 - asum;
    double th = 1.0;
#pragma unroll
    for (int k = 0; k < N; ++k) th = fmin(th, lim_theta((double)node.al[k], at[k], P.eps_i_a));
    if (th < 1.0) {
#pragma unroll
        for (int k = 0; k < N - 1; ++k) V.al[k] = (1.0 - th) * node.al[k] + th * V.al[k];
        cnt += cnt_one(C_ALG2);
    }
    // hard switch, judged on the completed limited state
    complete_from_prim<N, D, R>(e, V);
    bool hs = !isfinite(V.rc2) || !isfinite(V.p);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        hs |= !isfinite(V.ar[k]) || !isfinite(V.al[k]);
        hs |= (double)V.ar[k] < fmin(P.hs_i_ar, (double)node.ar[k]);
        hs |= (double)V.al[k] < fmin(P.hs_i_a, (double)node.al[k]);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) hs |= !isfinite(V.u[d]);
    hs |= (double)V.rc2 < fmin(P.hs_i_rc2, (double)node.rc2);
    if (hs) {
#pragma unroll
        for (int k = 0; k < N; ++k) V.ar[k] = node.ar[k];
#pragma unroll
        for (int d = 0; d < D; ++d) V.u[d] = node.u[d];
        V.p = node.p;
#pragma unroll
        for (int k = 0; k < N - 1; ++k) V.al[k] = node.al[k];
        complete_from_prim<N, D, R>(e, V);
        cnt += cnt_one(C_IHS);
    }
}

// all N volume fractions of a conservative vector
template <int N, int D>
__device__ inline void alphas(const double* W, double* al)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        al[k] = W[N + D + 1 + k];
        s += al[k];
    }
    al[N - 1] = 1.0 - s;
}

// Sec. 4.3.2 flux limiter (Alg. 3, Alg. 4, hard switch) at the face between
// nodes L = i and R = i+1.  G pairs are given as the "-" vector (M slots)
// plus the alpha slots of the "+" vector (N-1); the other slots agree.
//   W_i^+     = W_i     - 2 lambda (G^- - F_i)
//   W_{i+1}^- = W_{i+1} + 2 lambda (G^+ - F_{i+1})
// True when the high-order pair's half-cell states (Sec. 4.3.2) are finite
// and at or above every flux-limiter bound: then theta = 1 in Alg. 3 and
// Alg. 4 whatever the first-order states are (b >= eps >= min(eps, a)), the
// hard switch cannot fire (eps >= eps^HS, checked at set-up), and the
// limited pair is the high-order one.  Meaningful only with
// P.fast_flux_limiter.
template <int N, int D, int DIR>
__device__ inline bool flux_limit_clean(const EosDev& e, const ParDev& P, const St<N, D>& L, const St<N, D>& R,
                                        double lam, const double* Gho, const double* Gho_p)
{
    constexpr int IE = N + D, IA = N + D + 1;
    if (!P.fast_flux_limiter) return false;
    // the half-cell states W+ (from node i) and W- (from node i+1) are formed
    // slot by slot and checked at once, with running sums for rho, rho q-bar,
    // |rho u|^2 and the volume fractions, instead of being held whole
    const double uL = L.u[DIR], uR = R.u[DIR];
    const double l2 = 2.0 * lam;
    bool ok = true;
    double rp = 0.0, rm = 0.0, qp = 0.0, qm = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double wp = L.ar[k] - l2 * (Gho[k] - L.ar[k] * uL);
        const double wm = R.ar[k] + l2 * (Gho[k] - R.ar[k] * uR);
        ok = ok && wp >= P.eps_f_ar && wm >= P.eps_f_ar && isfinite(Gho[k]) && isfinite(wp) && isfinite(wm);
        rp += wp;
        rm += wm;
        qp += wp * e.q[k];
        qm += wm * e.q[k];
    }
    double m2p = 0.0, m2m = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double wp = L.mom[d] - l2 * (Gho[N + d] - (L.mom[d] * uL + (d == DIR ? L.p : 0.0)));
        const double wm = R.mom[d] + l2 * (Gho[N + d] - (R.mom[d] * uR + (d == DIR ? R.p : 0.0)));
        ok = ok && isfinite(Gho[N + d]) && isfinite(wp) && isfinite(wm);
        m2p += wp * wp;
        m2m += wm * wm;
    }
    const double Ep = L.E - l2 * (Gho[IE] - (L.E + L.p) * uL);
    const double Em = R.E + l2 * (Gho[IE] - (R.E + R.p) * uR);
    ok = ok && isfinite(Gho[IE]) && isfinite(Ep) && isfinite(Em);
    double sp = 0.0, sm = 0.0;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        const double ap = L.al[k] - l2 * (Gho[IA + k] - 0.0);
        const double am = R.al[k] + l2 * (Gho_p[k] - 0.0);
        ok = ok && ap >= P.eps_f_a && am >= P.eps_f_a && isfinite(Gho[IA + k]) && isfinite(Gho_p[k]) &&
             isfinite(ap) && isfinite(am);
        sp += ap;
        sm += am;
    }
    ok = ok && 1.0 - sp >= P.eps_f_a && 1.0 - sm >= P.eps_f_a;
    // rho (e - qbar) of each half-cell state, as rhoe_tilde forms it
    const double rep = Ep - 0.5 * m2p / rp - qp, rem = Em - 0.5 * m2m / rm - qm;
    return ok && rep >= P.eps_f_re && rem >= P.eps_f_re && isfinite(rep) && isfinite(rem);
}

template <int N, int D, int DIR>
__device__ inline void flux_limit(const EosDev& e, const ParDev& P, const St<N, D>& L, const St<N, D>& R,
                                  double lam, const double* Gho, const double* Gho_p, const double* Glo,
                                  const double* Glo_p, double* G, double* Gp, unsigned& cnt)
{
    constexpr int M = 2 * N + D, IE = N + D, IA = N + D + 1;
    double WL[M], WR[M], FL[M], FR[M];
    const double uL = L.u[DIR], uR = R.u[DIR];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        WL[k] = L.ar[k];
        WR[k] = R.ar[k];
        FL[k] = L.ar[k] * uL;
        FR[k] = R.ar[k] * uR;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        WL[N + d] = L.mom[d];
        WR[N + d] = R.mom[d];
        FL[N + d] = L.mom[d] * uL + (d == DIR ? L.p : 0.0);
        FR[N + d] = R.mom[d] * uR + (d == DIR ? R.p : 0.0);
    }
    WL[IE] = L.E;
    WR[IE] = R.E;
    FL[IE] = (L.E + L.p) * uL;
    FR[IE] = (R.E + R.p) * uR;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        WL[IA + k] = L.al[k];
        WR[IA + k] = R.al[k];
        FL[IA + k] = 0.0;
        FR[IA + k] = 0.0;
    }
    const double l2 = 2.0 * lam;
    // half-cell states of the first-order pair (reference values)
    double Wp_lo[M], Wm_lo[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const double gp = c >= IA ? Glo_p[c - IA] : Glo[c];
        Wp_lo[c] = WL[c] - l2 * (Glo[c] - FL[c]);
        Wm_lo[c] = WR[c] + l2 * (gp - FR[c]);
    }
    double ap_lo[N], am_lo[N];
    alphas<N, D>(Wp_lo, ap_lo);
    alphas<N, D>(Wm_lo, am_lo);
    const double rep_lo = rhoe_tilde<N, D>(e, Wp_lo), rem_lo = rhoe_tilde<N, D>(e, Wm_lo);

    // Alg. 3
    double Wp[M], Wm[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const double gp = c >= IA ? Gho_p[c - IA] : Gho[c];
        Wp[c] = WL[c] - l2 * (Gho[c] - FL[c]);
        Wm[c] = WR[c] + l2 * (gp - FR[c]);
    }
    double th = 1.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        th = fmin(th, lim_theta(Wp_lo[k], Wp[k], P.eps_f_ar));
        th = fmin(th, lim_theta(Wm_lo[k], Wm[k], P.eps_f_ar));
    }
    {
        double ap[N], am[N];
        alphas<N, D>(Wp, ap);
        alphas<N, D>(Wm, am);
#pragma unroll
        for (int k = 0; k < N; ++k) {
            th = fmin(th, lim_theta(ap_lo[k], ap[k], P.eps_f_a));
            th = fmin(th, lim_theta(am_lo[k], am[k], P.eps_f_a));
        }
    }
    if (th < 1.0) cnt += cnt_one(C_ALG3);
    // When Alg. 3 leaves theta = 1, G* = G^ho and W* = W^ho exactly.  If Alg. 4
    // also gives 1 and everything is finite, the hard switch cannot fire
    // (eps >= eps^HS, checked at context creation), so G** = G^ho: return
    // without rebuilding the half-cell states twice more.
    if (P.fast_flux_limiter && th == 1.0) {
        const double rep = rhoe_tilde<N, D>(e, Wp), rem = rhoe_tilde<N, D>(e, Wm);
        const double t2 = fmin(lim_theta(rep_lo, rep, P.eps_f_re), lim_theta(rem_lo, rem, P.eps_f_re));
        bool fin = isfinite(rep) && isfinite(rem) && isfinite(rep_lo) && isfinite(rem_lo);
#pragma unroll
        for (int c = 0; c < M; ++c) fin = fin && isfinite(Gho[c]) && isfinite(Wp_lo[c]) && isfinite(Wm_lo[c]);
#pragma unroll
        for (int k = 0; k < N - 1; ++k) fin = fin && isfinite(Gho_p[k]);
        if (t2 == 1.0 && fin) {
#pragma unroll
            for (int c = 0; c < M; ++c) G[c] = Gho[c];
#pragma unroll
            for (int k = 0; k < N - 1; ++k) Gp[k] = Gho_p[k];
            return;
        }
    }
    double Gs[M], Gsp[N > 1 ? N - 1 : 1];
#pragma unroll
    for (int c = 0; c < M; ++c) Gs[c] = (1.0 - th) * Glo[c] + th * Gho[c];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) Gsp[k] = (1.0 - th) * Glo_p[k] + th * Gho_p[k];

    // Alg. 4
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const double gp = c >= IA ? Gsp[c - IA] : Gs[c];
        Wp[c] = WL[c] - l2 * (Gs[c] - FL[c]);
        Wm[c] = WR[c] + l2 * (gp - FR[c]);
    }
    const double th2 = fmin(lim_theta(rep_lo, rhoe_tilde<N, D>(e, Wp), P.eps_f_re),
                            lim_theta(rem_lo, rhoe_tilde<N, D>(e, Wm), P.eps_f_re));
    if (th2 < 1.0) cnt += cnt_one(C_ALG4);
#pragma unroll
    for (int c = 0; c < M; ++c) G[c] = (1.0 - th2) * Glo[c] + th2 * Gs[c];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) Gp[k] = (1.0 - th2) * Glo_p[k] + th2 * Gsp[k];

    // hard switch on the final half-cell states
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const double gp = c >= IA ? Gp[c - IA] : G[c];
        Wp[c] = WL[c] - l2 * (G[c] - FL[c]);
        Wm[c] = WR[c] + l2 * (gp - FR[c]);
    }
    bool hs = false;
#pragma unroll
    for (int c = 0; c < M; ++c) hs |= !isfinite(G[c]);
#pragma unroll
    for (int k = 0; k < N - 1; ++k) hs |= !isfinite(Gp[k]);
    double ap[N], am[N];
    alphas<N, D>(Wp, ap);
    alphas<N, D>(Wm, am);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        hs |= Wp[k] < fmin(P.hs_f_ar, Wp_lo[k]);
        hs |= Wm[k] < fmin(P.hs_f_ar, Wm_lo[k]);
        hs |= ap[k] < fmin(P.hs_f_a, ap_lo[k]);
        hs |= am[k] < fmin(P.hs_f_a, am_lo[k]);
    }
    const double rep = rhoe_tilde<N, D>(e, Wp), rem = rhoe_tilde<N, D>(e, Wm);
    hs |= !isfinite(rep) || !isfinite(rem);
    hs |= rep < fmin(P.hs_f_re, rep_lo);
    hs |= rem < fmin(P.hs_f_re, rem_lo);
    if (hs) {
        cnt += cnt_one(C_FHS);
#pragma unroll
        for (int c = 0; c < M; ++c) G[c] = Glo[c];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) Gp[k] = Glo_p[k];
    }
}

constexpr int BC_PERIODIC = 1, BC_DIRICHLET = 2;

// ghost index map: transmissive copies the edge cell, periodic wraps
// (Dirichlet ghosts are read from the boundary-state array instead)
__device__ inline int map_bc(int g, int n, int lo, int hi)
{
    if (g < 0) return lo == 1 ? ((g % n) + n) % n : 0;
    if (g >= n) return hi == 1 ? g % n : n - 1;
    return g;
}

// the packed counts of a thread (cnt_one), summed over the wave as below
__device__ inline void flush_counters(unsigned packed, unsigned long long* dst);

// sum each counter over the wave, one atomic per non-zero counter.  Most
// counters are zero on every lane of most waves: a ballot skips those (the
// branch is wave-uniform), and the others are summed in 32 bits (a lane's
// counts stay far below 2^26 per launch) by lane permutes.
__device__ inline void flush_counters(const unsigned* c, unsigned long long* dst)
{
    const int lane = __lane_id();
#pragma unroll
    for (int k = 0; k < C_N; ++k) {
        if (__ballot(c[k] != 0u) == 0ull) continue;
        int v = (int)c[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __builtin_amdgcn_ds_bpermute((lane ^ off) << 2, v);
        if (lane == 0) atomicAdd(&dst[k], (unsigned long long)(unsigned)v);
    }
}

__device__ inline void flush_counters(unsigned packed, unsigned long long* dst)
{
    if (__ballot(packed != 0u) == 0ull) return;
    unsigned c[C_N];
#pragma unroll
    for (int k = 0; k < C_N; ++k) c[k] = cnt_get(packed, k);
    flush_counters(c, dst);
}

// NaN-propagating max (a NaN anywhere makes the result NaN)
__device__ inline double nmax(double a, double b) { return a != a ? a : (b != b ? b : fmax(a, b)); }

// block-wide max of D values (blockDim.x a multiple of 64, <= 256); the
// result is valid in thread 0; sh holds >= 4 * D doubles
template <int D>
__device__ inline void block_max(double* m, double* sh)
{
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m[d] = nmax(m[d], __shfl_xor(m[d], off, 64));
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) sh[w * D + d] = m[d];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
#pragma unroll
            for (int d = 0; d < D; ++d) m[d] = nmax(m[d], sh[i * D + d]);
}

// Sec. 4.2 infinite-rate thermal relaxation of one cell (species 0 is the
// only stiffened gas): A p^2 + B p + C = 0 (eq:Ap_Bp_Cp_1..3), positive root
// (taken as 2C/(-B - sqrt) when B > 0), T from eq:T_relax_e.  relaxed_pT
// returns p* and T* from W[0 .. N+D] (false when rho(e - qbar) <= 0 or no
// positive root exists); relax_cell then sets alpha_k = alpha_k rho_k /
// rho_k(p, T) for k < N-1, and leaves W unchanged where relaxed_pT fails.
// The root is ill-conditioned in a liquid at low pressure (its condition number
// grows like gamma_1 pinf_1 / p), so this function evaluates each formula in
// the order written, with IEEE division and no FMA contraction: its rounding
// is then reproducible by any plain double-precision evaluation of the same
// formulas.
template <int N, int D>
__device__ inline bool relaxed_pT(const EosDev& e, const double* W, double& p_out, double& T_out)
{
#pragma clang fp contract(off)
    constexpr int IE = N + D;
    double rho = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) rho += W[k];
    double cvb = 0.0, cpb = 0.0, qb = 0.0, Y0 = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double Y = W[k] / rho;  // mass fraction
        cvb += Y * e.cv[k];
        cpb += Y * e.g[k] * e.cv[k];
        qb += Y * e.q[k];
        if (k == 0) Y0 = Y;
    }
    double m2 = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) m2 += W[N + d] * W[N + d];
    const double re = W[IE] - 0.5 * m2 / rho - rho * qb;  // rho (e - qbar)
    if (!(re > 0.0) || !(rho > 0.0)) return false;
    const double p1 = e.pinf[0];
    const double R1 = e.g[0] * e.cv[0] - e.cv[0];  // c_p1 - c_v1
    const double A = cvb;
    const double B = -(re * (cpb - cvb) - p1 * cvb - p1 * Y0 * R1);
    const double C = -re * p1 * ((cpb - cvb) - Y0 * R1);
    const double disc = B * B - 4.0 * A * C;
    double p;
    if (B <= 0.0)
        p = (-B + sqrt(disc)) / (2.0 * A);
    else
        p = 2.0 * C / (-B - sqrt(disc));
    if (!(p > 0.0) || !isfinite(p)) return false;
    const double e_t = re / rho;
    const double T = e_t / (Y0 * (p + e.g[0] * p1) * e.cv[0] / (p + p1) + cvb - Y0 * e.cv[0]);
    if (!(T > 0.0) || !isfinite(T)) return false;
    p_out = p;
    T_out = T;
    return true;
}

template <int N, int D>
__device__ inline bool relax_cell(const EosDev& e, double* W)
{
#pragma clang fp contract(off)
    constexpr int IA = N + D + 1;
    double p, T;
    if (!relaxed_pT<N, D>(e, W, p, T)) return false;
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        const double rk = (p + e.pinf[k]) / ((e.g[k] - 1.0) * e.cv[k] * T);  // rho_k(p, T)
        W[IA + k] = W[k] / rk;
    }
    return true;
}

// Sec. 3: pressure and sound speed of the four-equation HRM from
// alpha_k rho_k, rho u and E.  p is the relaxed p* (eq:p_relax).  c^2 of
// eq:4_eqn_sos takes Psi_k and Gamma from the implicit derivative of the
// relaxation quadratic; scaled by rho it reads F(p) = S_v p^2 + B' p + C' with
//   S_v = sum m_k c_vk,  S_R = sum m_k (c_pk - c_vk),  S_2 = S_R - m_1 (c_p1 - c_v1),
//   B' = -(re S_R - pinf_1 S_v - pinf_1 m_1 (c_p1 - c_v1)),  C' = -re pinf_1 S_2,
// re = rho (e - qbar) = sum m_k (e - q_k) and m_k = alpha_k rho_k.  Summing
// Y_k dF/dm_k and using F(p) = 0 gives sum Y_k Psi_k = (re/rho) X and
// Gamma = X with X = (S_R p + pinf_1 S_2) / F'(p); and F'(p) = 2 S_v p + B' =
// S_v p - C'/p.  So
//   c^2 = p (re + p) (S_R p + pinf_1 S_2) / (rho (S_v p^2 + re pinf_1 S_2)),
// a quotient of positive terms (no cancellation, unlike 2 A_p p + B_p).
// p = c = NaN outside the admissible set.
template <int N, int D>
__device__ inline void hrm4_pc(const EosDev& e, const St<N, D>& s, double& p, double& c)
{
    double w[N + D + 1];
#pragma unroll
    for (int k = 0; k < N; ++k) w[k] = s.ar[k];
#pragma unroll
    for (int d = 0; d < D; ++d) w[N + d] = s.mom[d];
    w[N + D] = s.E;
    double T;
    if (!relaxed_pT<N, D>(e, w, p, T)) {
        p = c = __builtin_nan("");
        return;
    }
    double rho = 0.0, Sv = 0.0, SR = 0.0, rq = 0.0, m2 = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        rho += s.ar[k];
        Sv += s.ar[k] * e.cv[k];
        SR += s.ar[k] * (e.cp[k] - e.cv[k]);
        rq += s.ar[k] * e.q[k];
    }
#pragma unroll
    for (int d = 0; d < D; ++d) m2 += s.mom[d] * s.mom[d];
    const double re = s.E - 0.5 * m2 / rho - rq;
    const double S2 = SR - s.ar[0] * (e.cp[0] - e.cv[0]);
    const double p1 = e.pinf[0];
    c = sqrt(p * (re + p) * (SR * p + p1 * S2) / (rho * (Sv * p * p + re * p1 * S2)));
}

// First-order HLLC for the four-equation HRM solved directly, in direction
// DIR: the solver of Sec. 4.1.1 on (alpha_k rho_k, rho u, E) with the HRM
// pressure and sound speed of hrm4_pc, the same wave-speed estimates and
// sign(0) = 0.  The volume-fraction slots of G are zero.
template <int N, int D, int DIR>
__device__ inline void hllc4(const EosDev& e, const St<N, D>& L, const St<N, D>& Rs, double* G)
{
    constexpr int IE = N + D, IA = N + D + 1;
    double pL, cL, pR, cR;
    hrm4_pc<N, D>(e, L, pL, cL);
    hrm4_pc<N, D>(e, Rs, pR, cR);
    const double uL = L.u[DIR], uR = Rs.u[DIR];
    const double ub = 0.5 * (uL + uR), cb = 0.5 * (cL + cR);
    const double sL = fmin(ub - cb, uL - cL);
    const double sR = fmax(ub + cb, uR + cR);
    const double dL = sL - uL, dR = sR - uR;
    const double ss = (pR - pL + L.rho * uL * dL - Rs.rho * uR * dR) / (L.rho * dL - Rs.rho * dR);
    const double sg = ss > 0.0 ? 1.0 : (ss < 0.0 ? -1.0 : 0.0);
    const double wl = 0.5 * (1.0 + sg), wr = 0.5 * (1.0 - sg);
    const double sm = fmin(0.0, sL), sp = fmax(0.0, sR);
    const double chiL = dL / (sL - ss), chiR = dR / (sR - ss);
#pragma unroll
    for (int k = 0; k < N; ++k)
        G[k] = wl * (L.ar[k] * uL + sm * (chiL * L.ar[k] - L.ar[k])) +
               wr * (Rs.ar[k] * uR + sp * (chiR * Rs.ar[k] - Rs.ar[k]));
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double FLd = L.mom[d] * uL + (d == DIR ? pL : 0.0);
        const double FRd = Rs.mom[d] * uR + (d == DIR ? pR : 0.0);
        const double WsL = d == DIR ? chiL * L.rho * ss : chiL * L.rho * L.u[d];
        const double WsR = d == DIR ? chiR * Rs.rho * ss : chiR * Rs.rho * Rs.u[d];
        G[N + d] = wl * (FLd + sm * (WsL - L.mom[d])) + wr * (FRd + sp * (WsR - Rs.mom[d]));
    }
    const double EsL = chiL * (L.E + (ss - uL) * (L.rho * ss + pL / dL));
    const double EsR = chiR * (Rs.E + (ss - uR) * (Rs.rho * ss + pR / dR));
    G[IE] = wl * ((L.E + pL) * uL + sm * (EsL - L.E)) + wr * ((Rs.E + pR) * uR + sp * (EsR - Rs.E));
#pragma unroll
    for (int k = 0; k < N - 1; ++k) G[IA + k] = 0.0;
}

}  // namespace hrm
