// hrm_face.hpp -- one midpoint i+1/2 of the PP-WCNS-IS hyperbolic operator
// (arXiv:2208.04488 Sec. 4.1.1, Sec. 4.3, App. C, App. D), evaluated by one
// thread from the primitive data of the six nodes i-2..i+3 staged in LDS.
#pragma once

#include "hrm_device.hpp"

namespace hrm {

// LDS node record: the conservative vector W (M slots), then u_d (D),
// p, rho, c, rho c^2.
template <int N, int D>
struct NodeFields {
    static constexpr int M = 2 * N + D;
    static constexpr int U = M, P = M + D, RHO = M + D + 1, C = M + D + 2, RC2 = M + D + 3;
    static constexpr int COUNT = M + D + 4;
};

// node j of the stencil, field f; NS = LDS stride between consecutive nodes,
// FS = stride between fields
template <int NS, int FS>
__device__ inline double nodev(const double* nd, int j, int f)
{
    return nd[j * NS + f * FS];
}

template <int N, int D, int NS, int FS>
__device__ inline void load_node(const double* nd, int j, St<N, D>& s)
{
    using F = NodeFields<N, D>;
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
    s.rho = nodev<NS, FS>(nd, j, F::RHO);
    s.c = nodev<NS, FS>(nd, j, F::C);
    s.rc2 = nodev<NS, FS>(nd, j, F::RC2);
}

// left- and right-biased WENO-IS of one characteristic field given on the
// six stencil nodes; the right-biased value mirrors the stencil (App. C)
__device__ inline void weno_pair(const double* v, double eps, double& l, double& r)
{
    l = weno_is(v[0], v[1], v[2], v[3], v[4], eps);
    r = weno_is(v[5], v[4], v[3], v[2], v[1], eps);
}

// Output: G = G^{**,-}_{i+1/2} (M slots) and Gp = alpha slots of G^{**,+}.
template <int N, int D, int DIR, int NS, int FS>
__device__ void face_flux(const double* nd, const EosDev& e, const ParDev& P, double lam, double* G, double* Gp,
                          unsigned* cnt)
{
    using F = NodeFields<N, D>;
    constexpr int M = 2 * N + D, IE = N + D, IA = N + D + 1;
    constexpr int NA = N > 1 ? N - 1 : 1;

    St<N, D> L, R;
    load_node<N, D, NS, FS>(nd, 2, L);
    load_node<N, D, NS, FS>(nd, 3, R);

    // first-order HLLC of the node pair and its quasi-conservative pair (eq:G_pm)
    double Glo[M], Glo_p[NA];
    const double sslo = hllc<N, D, DIR>(L, R, Glo);
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        Glo_p[k] = Glo[IA + k] - sslo * R.al[k];
        Glo[IA + k] = Glo[IA + k] - sslo * L.al[k];
    }
    if (P.flags & F_FIRST_ORDER) {
#pragma unroll
        for (int c = 0; c < M; ++c) G[c] = Glo[c];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) Gp[k] = Glo_p[k];
        return;
    }

    // App. D: projection with the midpoint means of alpha_k rho_k, rho and c
    double arb[N];
#pragma unroll
    for (int k = 0; k < N; ++k) arb[k] = 0.5 * (L.ar[k] + R.ar[k]);
    const double rb = 0.5 * (L.rho + R.rho), cb = 0.5 * (L.c + R.c);
    const double irc = 1.0 / (rb * cb), irc2 = irc / cb;
    const double eps = P.eps_weno;
    double UL[M], UR[M], v[6];
#pragma unroll
    for (int j = 0; j < 6; ++j)
        v[j] = nodev<NS, FS>(nd, j, F::U + DIR) - nodev<NS, FS>(nd, j, F::P) * irc;
    weno_pair(v, eps, UL[0], UR[0]);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double s = arb[k] * irc2;
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] = nodev<NS, FS>(nd, j, k) - s * nodev<NS, FS>(nd, j, F::P);
        weno_pair(v, eps, UL[1 + k], UR[1 + k]);
    }
    {
        int t = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (d == DIR) continue;
#pragma unroll
            for (int j = 0; j < 6; ++j) v[j] = nodev<NS, FS>(nd, j, F::U + d);
            weno_pair(v, eps, UL[1 + N + t], UR[1 + N + t]);
            ++t;
        }
    }
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] = nodev<NS, FS>(nd, j, IA + k);
        weno_pair(v, eps, UL[N + D + k], UR[N + D + k]);
    }
#pragma unroll
    for (int j = 0; j < 6; ++j)
        v[j] = nodev<NS, FS>(nd, j, F::U + DIR) + nodev<NS, FS>(nd, j, F::P) * irc;
    weno_pair(v, eps, UL[M - 1], UR[M - 1]);

    // back to primitive slots: V = R U
    St<N, D> VL, VR;
    const double h2c = 0.5 / cb, hrc = 0.5 * rb * cb;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const double* U = side ? UR : UL;
        St<N, D>& V = side ? VR : VL;
        const double dU = U[M - 1] - U[0];
#pragma unroll
        for (int k = 0; k < N; ++k) V.ar[k] = U[1 + k] + arb[k] * h2c * dU;
        int t = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (d == DIR) {
                V.u[d] = 0.5 * (U[0] + U[M - 1]);
            } else {
                V.u[d] = U[1 + N + t];
                ++t;
            }
        }
        V.p = hrc * dU;
#pragma unroll
        for (int k = 0; k < N - 1; ++k) V.al[k] = U[N + D + k];
    }

    // Sec. 4.3.2 interpolation limiter: left against node i, right against node i+1
    if (!(P.flags & F_NO_LIMITERS)) {
        interp_limit<N, D>(e, P, VL, L, cnt);  // also completes the state
        interp_limit<N, D>(e, P, VR, R, cnt);
    } else {
        complete_from_prim<N, D>(e, VL);
        complete_from_prim<N, D>(e, VR);
    }

    // midpoint flux and velocity from HLLC on the interpolated states
    double Gt[M];
    const double ut = hllc<N, D, DIR>(VL, VR, Gt);

    // shock sensor (Sec. 4.3.1) on mixture density and pressure
    double sig = 0.0;
    if (!(P.flags & F_NO_BLEND)) {
        double r[6], pr[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            r[j] = nodev<NS, FS>(nd, j, F::RHO);
            pr[j] = nodev<NS, FS>(nd, j, F::P);
        }
        const double sr = 0.5 * (sensor_ratio(r[1], r[2], r[3], r[4], r[5]) + sensor_ratio(r[0], r[1], r[2], r[3], r[4]));
        const double sp = 0.5 * (sensor_ratio(pr[1], pr[2], pr[3], pr[4], pr[5]) +
                                 sensor_ratio(pr[0], pr[1], pr[2], pr[3], pr[4]));
        const double z = sr * sp;
        const double arg = P.Cs * (P.qexp == 2.0 ? z * z : pow(z, P.qexp));
        // tanh is exactly 0 at 0 and rounds to 1 for arguments >= 22
        sig = arg == 0.0 ? 0.0 : (arg >= 22.0 ? 1.0 : tanh(arg));
    }

    // HCS reconstruction (eq:reconstructed_G, eq:reconstructed_vel) and blending
    const double psi = P.psi, ha = P.hcs_a, hb = P.hcs_b, hc = P.hcs_c;
    double un[6], pj[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        un[j] = nodev<NS, FS>(nd, j, F::U + DIR);
        pj[j] = nodev<NS, FS>(nd, j, F::P);
    }
    double Gho[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        double g[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double w = nodev<NS, FS>(nd, j, c);
            if (c >= N && c < N + D)
                g[j] = w * un[j] + (c - N == DIR ? pj[j] : 0.0);
            else if (c == IE)
                g[j] = (w + pj[j]) * un[j];
            else
                g[j] = w * un[j];
        }
        const double ghcs = psi * Gt[c] - ha * (g[2] + g[3]) + hb * (g[1] + g[4]) - hc * (g[0] + g[5]);
        Gho[c] = sig * Gt[c] + (1.0 - sig) * ghcs;
    }
    const double uhcs = psi * ut - ha * (un[2] + un[3]) + hb * (un[1] + un[4]) - hc * (un[0] + un[5]);
    const double uh = sig * ut + (1.0 - sig) * uhcs;

    // high-order quasi-conservative pair: alpha slots minus u-hat alpha_i / alpha_{i+1}
    double Gho_p[NA];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        Gho_p[k] = Gho[IA + k] - uh * R.al[k];
        Gho[IA + k] = Gho[IA + k] - uh * L.al[k];
    }
    if (P.flags & F_NO_LIMITERS) {
#pragma unroll
        for (int c = 0; c < M; ++c) G[c] = Gho[c];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) Gp[k] = Gho_p[k];
        return;
    }
    flux_limit<N, D, DIR>(e, P, L, R, lam, Gho, Gho_p, Glo, Glo_p, G, Gp, cnt);
}

}  // namespace hrm
