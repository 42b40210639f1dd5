// hrm_face.hpp -- one midpoint i+1/2 of the PP-WCNS-IS hyperbolic operator
// (arXiv:2208.04488 Sec. 4.1.1, Sec. 4.3, App. C, App. D), evaluated by one
// thread from the primitive data of the six nodes i-2..i+3 staged in LDS.
#pragma once

#include "hrm_device.hpp"
#include "hrm_mlp.hpp"

namespace hrm {

// LDS node record: the conservative vector W (M slots), then u_d (D),
// p, rho, c, rho c^2.  The slim record leaves rho out (it is the sum of the
// partial densities, formed again where it is read): one field less lets
// the 3D y- and z-sweeps' 16 x 16 tiles fit four workgroups per CU.
template <int N, int D, bool SLIM = false>
struct NodeFields {
    static constexpr int M = 2 * N + D;
    static constexpr bool slim = SLIM;
    static constexpr int U = M, P = M + D, RHO = SLIM ? -1 : M + D + 1;
    static constexpr int C = M + D + (SLIM ? 1 : 2), RC2 = C + 1;
    static constexpr int COUNT = RC2 + 1;
};

// node j of the stencil, field f; NS = LDS stride between consecutive nodes,
// FS = stride between fields
template <int NS, int FS>
__device__ inline double nodev(const double* nd, int j, int f)
{
    return nd[j * NS + f * FS];
}

// mixture density of node j: read, or in the slim record the sum of the
// partial densities in the order the staging pass forms it (the same bits)
template <class F, int N, int NS, int FS>
__device__ inline double node_rho(const double* nd, int j)
{
    if constexpr (F::slim) {
        double r = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) r += nodev<NS, FS>(nd, j, k);
        return r;
    } else {
        return nodev<NS, FS>(nd, j, F::RHO);
    }
}

template <int N, int D, int NS, int FS, bool SLIM>
__device__ inline void load_node(const double* nd, int j, St<N, D>& s)
{
    using F = NodeFields<N, D, SLIM>;
    constexpr int IE = N + D, IA = N + D + 1;
    double asum = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) s.ar[k] = nodev<NS, FS>(nd, j, k);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        s.mom[d] = nodev<NS, FS>(nd, j, N + d);
        s.u[d] = nodev<NS, FS>(nd, j, F::U + d);
    }
    s.E = nodev<NS, FS>(nd, j, IE);
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        s.al[k] = nodev<NS, FS>(nd, j, IA + k);
        asum += s.al[k];
    }
    s.al[N - 1] = 1.0 - asum;
    s.p = nodev<NS, FS>(nd, j, F::P);
    s.rho = node_rho<F, N, NS, FS>(nd, j);
    s.c = nodev<NS, FS>(nd, j, F::C);
    s.rc2 = nodev<NS, FS>(nd, j, F::RC2);
}

// left- and right-biased WENO-IS of one characteristic field given on the
// six stencil nodes; the right-biased value mirrors the stencil (App. C)
template <typename R>
__device__ inline void weno_pair(const R* v, double eps, R& l, R& r)
{
    weno_is_pair<R>(v, eps, l, r);
}

// the pair of interpolated values at i+1/2 from v[0..5] = nodes i-2..i+3:
// App. C weights (WT = 0), or the learned weights (WT = 1) with App. C as the
// fallback where a learned weight is not finite.  WT = 1 must be reached by
// every lane of the wave (matrix-core evaluation).
template <typename R, int WT>
__device__ inline void interp_pair(const R* v, double eps, const MlpPacked* mlp, R& l, R& r)
{
    if constexpr (WT == 0) {
        weno_pair<R>(v, eps, l, r);
    } else {
        const R ul[5] = {v[0], v[1], v[2], v[3], v[4]};
        const R ur[5] = {v[5], v[4], v[3], v[2], v[1]};
        float xl[5], xr[5], zl[3], zr[3], wl[3], wr[3];
        mlp_inputs<R>(ul, xl);
        mlp_inputs<R>(ur, xr);
        mlp_logits(mlp, xl, zl);
        mlp_logits(mlp, xr, zr);
        l = mlp_omega(zl, xl, wl) ? mlp_value<R>(ul, wl) : weno_is<R>(v[0], v[1], v[2], v[3], v[4], eps);
        r = mlp_omega(zr, xr, wr) ? mlp_value<R>(ur, wr) : weno_is<R>(v[5], v[4], v[3], v[2], v[1], eps);
    }
}

// normalised fourth-order second derivative of the shock sensor (Sec. 4.3.1)
template <typename R>
__device__ inline R sensor_ratio_t(R v0, R v1, R v2, R v3, R v4)
{
    const R num = fabs(-v0 + (R)16 * v1 - (R)30 * v2 + (R)16 * v3 - v4);
    const R den = fabs(v0 + (R)16 * v1 + (R)30 * v2 + (R)16 * v3 + v4);
    if constexpr (sizeof(R) == sizeof(double))
        if (den > 1e-290) return num * rcp_newton(den);  // densities and pressures: far from subnormal
    return den > (R)0 ? num / den : (num > (R)0 ? (R)1 : (R)0);
}

// Output: G = G^{**,-}_{i+1/2} (M slots) and Gp = alpha slots of G^{**,+}.
// R is the face arithmetic type; node data, the flux limiter and the outputs
// are double.  LOW = false leaves out the first-order and direct-HRM branches
// (selected by flags) for callers that never take them.  Always inlined:
// a call would spill the whole face state around it.
template <int N, int D, int DIR, int NS, int FS, typename R, int WT = 0, bool LOW = true, bool SLIM = false>
__device__ __forceinline__ void face_flux(const double* nd, const EosDev& e, const ParDev& P, double lam, double* G, double* Gp,
                          unsigned& cnt)
{
    static_assert(2 * N <= 15, "per-face counts are packed 4 bits per counter");
    using F = NodeFields<N, D, SLIM>;
    constexpr int M = 2 * N + D, IE = N + D, IA = N + D + 1;
    constexpr int NA = N > 1 ? N - 1 : 1;
    // FP32: the characteristic fields are interpolated as deviations from
    // node i, formed in double.  WENO-IS is translation-equivariant (the
    // smoothness indicators use differences only and the candidate weights
    // sum to one), so this is the same interpolation, but float now resolves
    // the small differences u +- p/(rho c) that carry the pressure in a liquid.
    constexpr bool DELTA = sizeof(R) != sizeof(double);
    auto nv = [&](int j, int f) -> R { return (R)nodev<NS, FS>(nd, j, f); };
    auto dv = [&](int j, int f) -> R {
        return DELTA ? (R)(nodev<NS, FS>(nd, j, f) - nodev<NS, FS>(nd, 2, f)) : (R)nodev<NS, FS>(nd, j, f);
    };
    auto back = [&](int f, R d) -> R { return DELTA ? (R)(nodev<NS, FS>(nd, 2, f) + (double)d) : d; };
    auto back_d = [&](int f, R d) -> double { return DELTA ? nodev<NS, FS>(nd, 2, f) + (double)d : (double)d; };

    // the two nodes of the face (i, i+1), read from LDS where they are used:
    // the compiler barrier forces fresh reads, so the node states do not
    // occupy registers across the whole face computation
    auto node_pair = [&](St<N, D>& a, St<N, D>& b) {
        asm volatile("" ::: "memory");
        load_node<N, D, NS, FS, SLIM>(nd, 2, a);
        load_node<N, D, NS, FS, SLIM>(nd, 3, b);
    };

    // first-order HLLC of the node pair and its quasi-conservative pair
    // (eq:G_pm); needed only by the first-order scheme and by the flux
    // limiter when it has to act, so it is formed on demand
    auto first_order = [&](const St<N, D>& L, const St<N, D>& Rn, double* Glo, double* Glo_p) {
        const St<N, D, R> Lr = convert<N, D, R>(L), Rr = convert<N, D, R>(Rn);
        const double ss = hllc<N, D, DIR, R>(Lr, Rr, Glo);
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
            Glo_p[k] = Glo[IA + k] - ss * Rr.al[k];
            Glo[IA + k] = Glo[IA + k] - ss * Lr.al[k];
        }
    };
    if (LOW && (P.flags & F_FIRST_ORDER)) {
        St<N, D> L, Rn;
        node_pair(L, Rn);
        if (P.flags & F_FOUR_EQ) {
            hllc4<N, D, DIR>(e, L, Rn, G);
#pragma unroll
            for (int k = 0; k < N - 1; ++k) Gp[k] = 0.0;
            return;
        }
        double Glo[M], Glo_p[NA];
        first_order(L, Rn, Glo, Glo_p);
#pragma unroll
        for (int c = 0; c < M; ++c) G[c] = Glo[c];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) Gp[k] = Glo_p[k];
        return;
    }

    // App. D: projection with the midpoint means of alpha_k rho_k, rho and c
    R arb[N];
#pragma unroll
    for (int k = 0; k < N; ++k) arb[k] = (R)0.5 * (nv(2, k) + nv(3, k));
    const R rb = (R)0.5 * ((R)node_rho<F, N, NS, FS>(nd, 2) + (R)node_rho<F, N, NS, FS>(nd, 3));
    const R cb = (R)0.5 * (nv(2, F::C) + nv(3, F::C));
    // 1/(rho c), 1/(rho c^2) = rho (1/(rho c))^2 and 1/(2c) = rho/(2 rho c) from one
    // reciprocal (the means of two admissible nodes are positive)
    R irc;
    if constexpr (sizeof(R) == sizeof(double))
        irc = rcp_newton(rb * cb);
    else
        irc = (R)1 / (rb * cb);
    const R irc2 = irc * irc * rb;
    const double eps = P.eps_weno;
    // The characteristic fields are interpolated one at a time and each is
    // taken back to its primitive slot (V = R U) at once, so that only the
    // two acoustic fields stay live across the others.
    St<N, D, R> VL, VR;
    const R h2c = (R)0.5 * rb * irc, hrc = (R)0.5 * rb * cb;
    R v[6], aL0, aR0, aLM, aRM;
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] = dv(j, F::U + DIR) - dv(j, F::P) * irc;
    interp_pair<R, WT>(v, eps, P.mlp, aL0, aR0);
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] = dv(j, F::U + DIR) + dv(j, F::P) * irc;
    interp_pair<R, WT>(v, eps, P.mlp, aLM, aRM);
    const R dUL = aLM - aL0, dUR = aRM - aR0;
    VL.u[DIR] = back(F::U + DIR, (R)0.5 * (aL0 + aLM));
    VR.u[DIR] = back(F::U + DIR, (R)0.5 * (aR0 + aRM));
    VL.p = back(F::P, hrc * dUL);
    VR.p = back(F::P, hrc * dUR);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const R s = arb[k] * irc2;
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] = dv(j, k) - s * dv(j, F::P);
        R l, r;
        interp_pair<R, WT>(v, eps, P.mlp, l, r);
        VL.ar[k] = back(k, l + arb[k] * h2c * dUL);
        VR.ar[k] = back(k, r + arb[k] * h2c * dUR);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if (d == DIR) continue;
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] = dv(j, F::U + d);
        R l, r;
        interp_pair<R, WT>(v, eps, P.mlp, l, r);
        VL.u[d] = back(F::U + d, l);
        VR.u[d] = back(F::U + d, r);
    }
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] = dv(j, IA + k);
        R l, r;
        interp_pair<R, WT>(v, eps, P.mlp, l, r);
        VL.al[k] = back_d(IA + k, l);
        VR.al[k] = back_d(IA + k, r);
    }

    // Sec. 4.3.2 interpolation limiter: left against node i, right against node i+1
    if (!(P.flags & F_NO_LIMITERS)) {
        St<N, D> L, Rn;
        node_pair(L, Rn);
        interp_limit<N, D, R>(e, P, VL, convert<N, D, R>(L), cnt);  // also completes the state
        interp_limit<N, D, R>(e, P, VR, convert<N, D, R>(Rn), cnt);
    } else {
        complete_from_prim<N, D, R>(e, VL);
        complete_from_prim<N, D, R>(e, VR);
    }

    // midpoint flux and velocity from HLLC on the interpolated states
    double Gt[M];
    const R ut = hllc<N, D, DIR, R>(VL, VR, Gt);

    // shock sensor (Sec. 4.3.1) on mixture density and pressure, in double in
    // both variants: C_s = 1e12 turns float rounding of p at a contact into
    // a visible blending weight
    R sig = 0;
    if (!(P.flags & F_NO_BLEND)) {
        double r[6], pr[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            r[j] = node_rho<F, N, NS, FS>(nd, j);
            pr[j] = nodev<NS, FS>(nd, j, F::P);
        }
        const double sr = 0.5 * (sensor_ratio_t<double>(r[1], r[2], r[3], r[4], r[5]) +
                                 sensor_ratio_t<double>(r[0], r[1], r[2], r[3], r[4]));
        const double sp = 0.5 * (sensor_ratio_t<double>(pr[1], pr[2], pr[3], pr[4], pr[5]) +
                                 sensor_ratio_t<double>(pr[0], pr[1], pr[2], pr[3], pr[4]));
        const double z = sr * sp;
        const double arg = P.Cs * (P.qexp == 2.0 ? z * z : pow(z, P.qexp));
        // tanh is exactly 0 at 0 and rounds to 1 for arguments >= 22; below
        // 0.01 (smooth flow: nearly every face) its odd series to x^7 is
        // exact to double rounding (the next term is below 3e-18 x)
        double th;
        if (arg < 0.01) {
            const double a2 = arg * arg;
            th = arg * (1.0 + a2 * (-1.0 / 3.0 + a2 * (2.0 / 15.0 - a2 * (17.0 / 315.0))));
        } else {
            th = arg >= 22.0 ? 1.0 : tanh(arg);
        }
        sig = (R)th;
    }

    // HCS reconstruction (eq:reconstructed_G, eq:reconstructed_vel) and blending.
    // Volume-fraction slots and the face velocity u-hat are double in both
    // variants: G^+-_alpha = G_alpha - u-hat alpha_i cancels to (alpha-tilde -
    // alpha_i) u-hat only if both terms see the same velocity at full precision.
    const R psi = (R)P.psi, ha = (R)P.hcs_a, hb = (R)P.hcs_b, hc = (R)P.hcs_c;
    const double psid = P.psi, had = P.hcs_a, hbd = P.hcs_b, hcd = P.hcs_c;
    R un[6], pj[6];
    double und[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        und[j] = nodev<NS, FS>(nd, j, F::U + DIR);
        un[j] = (R)und[j];
        pj[j] = nv(j, F::P);
    }
    double Gho[M], Gho_p[NA];
    const double sigd = sig;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        if (c >= IA) {
            double g[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) g[j] = nodev<NS, FS>(nd, j, c) * und[j];
            const double ghcs = psid * Gt[c] - had * (g[2] + g[3]) + hbd * (g[1] + g[4]) - hcd * (g[0] + g[5]);
            Gho[c] = sigd * Gt[c] + (1.0 - sigd) * ghcs;
        } else {
            R g[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const R w = nv(j, c);
                if (c >= N && c < N + D)
                    g[j] = w * un[j] + (c - N == DIR ? pj[j] : (R)0);
                else if (c == IE)
                    g[j] = (w + pj[j]) * un[j];
                else
                    g[j] = w * un[j];
            }
            const R gt = (R)Gt[c];
            const R ghcs = psi * gt - ha * (g[2] + g[3]) + hb * (g[1] + g[4]) - hc * (g[0] + g[5]);
            Gho[c] = (double)(sig * gt + ((R)1 - sig) * ghcs);
        }
    }
    const double utd = ut;
    const double uhcs = psid * utd - had * (und[2] + und[3]) + hbd * (und[1] + und[4]) - hcd * (und[0] + und[5]);
    const double uh = sigd * utd + (1.0 - sigd) * uhcs;

    // high-order quasi-conservative pair: alpha slots minus u-hat alpha_i / alpha_{i+1}
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        Gho_p[k] = Gho[IA + k] - uh * nodev<NS, FS>(nd, 3, IA + k);
        Gho[IA + k] = Gho[IA + k] - uh * nodev<NS, FS>(nd, 2, IA + k);
    }
    if (P.flags & F_NO_LIMITERS) {
#pragma unroll
        for (int c = 0; c < M; ++c) G[c] = Gho[c];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) Gp[k] = Gho_p[k];
        return;
    }
    // Alg. 3 and Alg. 4 leave the high-order pair untouched when its half-cell
    // states already satisfy every bound (the usual case away from
    // interfaces and shocks); the first-order pair is formed only otherwise
    St<N, D> L, Rn;
    node_pair(L, Rn);
    if (flux_limit_clean<N, D, DIR>(e, P, L, Rn, lam, Gho, Gho_p)) {
#pragma unroll
        for (int c = 0; c < M; ++c) G[c] = Gho[c];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) Gp[k] = Gho_p[k];
        return;
    }
    // In double, the full limiter reads the node pair afresh (the same
    // values): products of the check above are then not kept for it, and the
    // usual path carries no registers (spilled, at this pressure) into the
    // rare one.  256^3 FP64 step -4 %; the float variant, which spills less,
    // measured 1 % slower with it.
    St<N, D> Lf = L, Rf = Rn;
    if constexpr (sizeof(R) == sizeof(double)) node_pair(Lf, Rf);
    double Glo[M], Glo_p[NA];
    first_order(Lf, Rf, Glo, Glo_p);
    flux_limit<N, D, DIR>(e, P, Lf, Rf, lam, Gho, Gho_p, Glo, Glo_p, G, Gp, cnt);
}

}  // namespace hrm
