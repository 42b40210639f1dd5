// hrm.hip -- gfx950 kernels and the C-ABI of the PP-WCNS-IS stage and the
// thermal relaxation (arXiv:2208.04488).  Declarations and semantics of the
// exported calls are in include/hrm.h.
//
// Kernels
//   k_sweep<N,D,DIR>  one direction of the spatial operator.  A block stages
//                     the primitive data of a tile of nodes (with the 3-node
//                     halo on both sides, boundary conditions applied at load)
//                     in LDS, computes one face per thread, writes the face
//                     pairs back to LDS and forms the flux difference of each
//                     cell.  The last direction also applies the Shu-Osher
//                     stage update and, optionally, the relaxation; in the
//                     last stage of a step it also folds the block maxima
//                     of |u_d| + c of the new state into the partial slots
//                     of the next step's time step.
//   k_relax           point-wise relaxation.
//   k_wavespeed       per-block max of |u_d| + c (the first step of a run,
//                     hrm_max_wavespeed), then k_reduce_max / k_reduce_dt
//                     (which clears the slots the sweep folds into).
//   k_dt              the time step and lambda_d on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>

#include "hrm.h"
#include "hrm_face.hpp"

namespace hrm {

struct SweepArgs {
    const double* Ws;
    const double* Wn;
    double* Wout;
    double* rhs;
    const double* slot;
    unsigned long long* cnt;
    long long ncell;
    int n[3];
    int bclo, bchi;
    const double* blo;  // Dirichlet ghost states of the low / high face (M x face cells), or null
    const double* bhi;
    double* wpart;  // mode 2, non-null: maxima of |u_d| + c of the stage output, block b into slot b % nslot
    unsigned nslot; // a power of two, at most the number of blocks
    int mode;  // 0: rhs = L_d, 1: rhs += L_d, 2: stage update with rhs + L_d
    int relax;
    int hold;  // mode 2 within a full RK3 step: a step of dt = 0 (the end time reached) leaves W^n as it is
    double a, b;
    double idx;
    EosDev e;
    ParDev P;
};

constexpr int MODE_WRITE = 0, MODE_ADD = 1, MODE_FINAL = 2;

// one DPP move of a 64-bit value (both halves with the same control); rows
// outside ROWS keep their own value
template <int CTRL, int ROWS>
__device__ inline unsigned long long dpp_u64(unsigned long long v)
{
    const int lo = (int)(unsigned)v, hi = (int)(unsigned)(v >> 32);
    const int l = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    const int h = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
    return ((unsigned long long)(unsigned)h << 32) | (unsigned)l;
}

__device__ inline unsigned long long umax64(unsigned long long a, unsigned long long b) { return a > b ? a : b; }

// maximum of a 64-bit unsigned value over the wave (all 64 lanes active),
// returned in every lane: within each row of 16 lanes by quad permutes and
// mirrors, then across rows by the row broadcasts, read back from lane 63
__device__ inline unsigned long long wave_umax64(unsigned long long v)
{
    v = umax64(v, dpp_u64<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
    v = umax64(v, dpp_u64<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
    v = umax64(v, dpp_u64<0x141, 0xF>(v));  // row_half_mirror
    v = umax64(v, dpp_u64<0x140, 0xF>(v));  // row_mirror: row maximum in every lane
    v = umax64(v, dpp_u64<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
    v = umax64(v, dpp_u64<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// Tile: BS face threads along the sweep direction (BS-1 cells), BA threads
// across it.  DIR == 0: blockDim = (BS, BA), across = y, blockIdx.z = z.
// DIR == 1: blockDim = (BA, BS), across = x, blockIdx.z = z.
// DIR == 2: blockDim = (BA, BS), across = x, blockIdx.z = y.
// The tile index along the sweep is blockIdx.y (in 2D and 3D), so that
// tiles sharing a halo have linear block indices gridDim.x apart: on the
// same XCD (and L2) when gridDim.x is a multiple of 8, and dispatched close
// together; 1D keeps the tiles on blockIdx.x, the dimension with room for
// long lines.
// The register budget of the sweeps is cut to three waves per SIMD (168
// VGPRs): the third wave hides more LDS and memory latency than the spills
// it causes cost (1024 x 512 step 0.441 -> 0.400 ms, 256^3 FP64 +3 %, FP32
// +11 %).  A fourth wave (128 VGPRs) pays for the plain FP64 sweeps once the
// face keeps few values past the flux limiter's check, where the
// workgroups' LDS fits: 1024 x 512 step -1.9 %, 256^3 x-sweep -1.5 %,
// z-sweep (three arrays read per cell after its barriers) -5 %, y-sweep
// -2 %.  The 3D y- and z-sweeps' 16 x 16 tiles fit four workgroups per CU
// only with the slim node record (rho formed again where read, which costs
// the x-sweep 2 % where its LDS fits anyway).  In float a fourth wave does
// not pay (256^3 x-sweep +3.5 %).
template <int D, int DIR, typename R, int WT>
constexpr bool sweep_slim()
{
    return sizeof(R) == sizeof(double) && WT == 0 && D == 3 && DIR >= 1;
}

template <int D, int DIR, typename R, int WT>
constexpr int sweep_waves()
{
    return sizeof(R) == sizeof(double) && WT == 0 && D >= 2 ? 4 : 3;
}

// WS: the launch is a stage update that also folds the wavespeed maxima of
// its output into A.wpart; a separate instantiation, so that the other
// launches keep their register allocation
template <int N, int D, int DIR, int BS, int BA, typename R, int WT, bool WS = false>
__global__ void __launch_bounds__(BS* BA, (sweep_waves<D, DIR, R, WT>())) k_sweep(const SweepArgs A)
{
    constexpr bool SLIM = sweep_slim<D, DIR, R, WT>();
    using F = NodeFields<N, D, SLIM>;
    constexpr int M = 2 * N + D, IA = N + D + 1;
    constexpr int NA = N > 1 ? N - 1 : 1;
    constexpr int LN = BS + 5;
    constexpr int FS = BA * LN;
    constexpr int NS = DIR == 0 ? 1 : BA;
    static_assert((BS * BA) % 64 == 0, "whole waves");
    __shared__ double lds[F::COUNT * FS];

    const int ts = DIR == 0 ? threadIdx.x : threadIdx.y;
    const int ta = DIR == 0 ? threadIdx.y : threadIdx.x;
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const long long st[3] = {1, A.n[0], (long long)A.n[0] * A.n[1]};
    int c0, abase, other, adim, odim;
    if (DIR == 0) {
        c0 = (D == 1 ? blockIdx.x : blockIdx.y) * (BS - 1);
        abase = (D == 1 ? blockIdx.y : blockIdx.x) * BA;
        other = blockIdx.z;
        adim = 1;
        odim = 2;
    } else if (DIR == 1) {
        c0 = blockIdx.y * (BS - 1);
        abase = blockIdx.x * BA;
        other = blockIdx.z;
        adim = 0;
        odim = 2;
    } else {
        c0 = blockIdx.y * (BS - 1);
        abase = blockIdx.x * BA;
        other = blockIdx.z;
        adim = 0;
        odim = 1;
    }
    const int nsw = A.n[DIR], na = A.n[adim];
    const long long nc = A.ncell;
    auto base = [](int a, int l) { return DIR == 0 ? a * LN + l : l * BA + a; };

    // stage the node tile (sweep index c0-3 .. c0+BS+1) with its primitives.
    // The staging waves run at raised priority, so that a workgroup starting
    // beside others still computing faces gets its loads out first (1024 x
    // 512 step -2.4 %, 256^3 FP64 -1 %, FP32 -2.6 %; raising it also around
    // the stage update's loads measured slower)
    __builtin_amdgcn_s_setprio(3);
    for (int q = tid; q < LN * BA; q += BS * BA) {
        const int l = DIR == 0 ? q % LN : q / BA;
        const int a = DIR == 0 ? q / LN : q % BA;
        const int gi = c0 - 3 + l;
        const int ca = min(abase + a, na - 1);
        const double* src = A.Ws;
        long long idx, stride = nc;
        if ((gi < 0 && A.bclo == BC_DIRICHLET) || (gi >= nsw && A.bchi == BC_DIRICHLET)) {
            // Dirichlet: every ghost node takes the boundary state of its line
            src = gi < 0 ? A.blo : A.bhi;
            idx = ca + (long long)na * other;
            stride = (long long)na * A.n[odim];
        } else {
            idx = map_bc(gi, nsw, A.bclo, A.bchi) * st[DIR] + ca * st[adim] + other * st[odim];
        }
        double W[M];
#pragma unroll
        for (int c = 0; c < M; ++c) W[c] = src[c * stride + idx];
        St<N, D> s;
        state_from_W<N, D>(A.e, W, s);
        const int b = base(a, l);
#pragma unroll
        for (int c = 0; c < M; ++c) lds[c * FS + b] = W[c];
#pragma unroll
        for (int d = 0; d < D; ++d) lds[(F::U + d) * FS + b] = s.u[d];
        lds[F::P * FS + b] = s.p;
        if constexpr (!SLIM) lds[F::RHO * FS + b] = s.rho;
        lds[F::C * FS + b] = s.c;
        lds[F::RC2 * FS + b] = s.rc2;
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();

    // one face per thread: between sweep nodes c0-1+ts and c0+ts.  In the
    // z-sweep a wave holds four consecutive ts; one whose faces all lie
    // beyond face nsw (three waves of the last tile of a 256-cell line)
    // skips them and their LDS writes, which no cell reads (256^3 z-sweep
    // -1.3 %; the same skip in the y-sweeps and in 1D measured no better,
    // the branch costing them as much in register allocation)
    const bool live = DIR != 2 || c0 + __builtin_amdgcn_readfirstlane(tid >> 6) * (64 / BA) <= nsw;
    unsigned cnt = 0;  // packed counts (cnt_one)
    double G[M], Gp[NA];
    if (live) {
        unsigned lc = 0;
        face_flux<N, D, DIR, NS, FS, R, WT, true, SLIM>(lds + base(ta, ts), A.e, A.P, A.slot[1 + DIR], G, Gp, lc);
        // face c0+ts is counted once: the last face of a tile is the first
        // face of the next tile unless it is the boundary face nsw
        const int f = c0 + ts;
        const bool ok = f <= nsw && (ts < BS - 1 || f == nsw) && (abase + ta < na);
        if (ok) cnt = lc;
    }
    // A middle direction only adds to the right-hand side (MODE_ADD): its
    // cell's accumulated values are loaded here, before the barriers, so that
    // their latency overlaps the wait for the block's slowest face (3D
    // y-sweep -11 %; the other directions keep their loads where they are
    // used, which measured faster for them)
    constexpr bool MID = DIR > 0 && DIR < D - 1;
    double Rc[MID ? M : 1];
    if constexpr (MID) {
        const int ci = c0 + ts, ca = abase + ta;
        if (ts < BS - 1 && ci < nsw && ca < na) {
            const long long cell = ci * st[DIR] + ca * st[adim] + other * st[odim];
#pragma unroll
            for (int c = 0; c < M; ++c) Rc[c] = A.rhs[c * nc + cell];
        }
    }
    __syncthreads();
    if (live) {
        const int b = base(ta, ts);
#pragma unroll
        for (int c = 0; c < M; ++c) lds[c * FS + b] = G[c];
#pragma unroll
        for (int k = 0; k < N - 1; ++k) lds[(M + k) * FS + b] = Gp[k];
    }
    __syncthreads();

    // flux difference of cell c0+ts: faces ts (i-1/2) and ts+1 (i+1/2)
    const int ci = c0 + ts, ca = abase + ta;
    double wmax[D];
#pragma unroll
    for (int d = 0; d < D; ++d) wmax[d] = 0.0;
    if (ts < BS - 1 && ci < nsw && ca < na) {
        const long long cell = ci * st[DIR] + ca * st[adim] + other * st[odim];
        const int bl = base(ta, ts), br = base(ta, ts + 1);
        double L[M];
#pragma unroll
        for (int c = 0; c < IA; ++c) L[c] = -(lds[c * FS + br] - lds[c * FS + bl]) * A.idx;
#pragma unroll
        for (int k = 0; k < N - 1; ++k) L[IA + k] = -(lds[(IA + k) * FS + br] - lds[(M + k) * FS + bl]) * A.idx;
        if (A.mode == MODE_WRITE) {
#pragma unroll
            for (int c = 0; c < M; ++c) A.rhs[c * nc + cell] = L[c];
        } else if (A.mode == MODE_ADD) {
            if constexpr (MID) {
#pragma unroll
                for (int c = 0; c < M; ++c) A.rhs[c * nc + cell] = Rc[c] + L[c];
            } else {
#pragma unroll
                for (int c = 0; c < M; ++c) A.rhs[c * nc + cell] += L[c];
            }
        } else {
            const double dt = A.slot[0];
            double w[M];
            if (__builtin_expect(A.hold && dt == 0.0, 0)) {
                // every stage of a step of length 0 is W^n in exact arithmetic;
                // written as such, a run held at its end time stays bit for bit
#pragma unroll
                for (int c = 0; c < M; ++c) w[c] = A.Wn[c * nc + cell];
            } else {
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    const double Lc = D > 1 ? A.rhs[c * nc + cell] + L[c] : L[c];
                    w[c] = A.a * A.Wn[c * nc + cell] + A.b * (A.Ws[c * nc + cell] + dt * Lc);
                }
                if (A.relax && !relax_cell<N, D>(A.e, w)) cnt += cnt_one(C_RELAX_BAD);
            }
#pragma unroll
            for (int c = 0; c < M; ++c) A.Wout[c * nc + cell] = w[c];
            if constexpr (WS) {
                // Sec. 4.1.2: |u_d| + c of the new state, for the next time step
                St<N, D> s;
                state_from_W<N, D>(A.e, w, s);
                double cs = s.c;
                if (A.P.flags & F_FOUR_EQ) {
                    double p;
                    hrm4_pc<N, D>(A.e, s, p, cs);
                }
#pragma unroll
                for (int d = 0; d < D; ++d) wmax[d] = fabs(s.u[d]) + cs;
            }
        }
    }
    if constexpr (WS) {
        // wave maximum, folded into slot (linear block index) % nslot, which
        // the time-step reduction has cleared.  The values are +0 or above,
        // or NaN; their bit patterns order as unsigned integers the same way,
        // with every NaN above every number, so the maximum is taken on the
        // bits: without branches, and by the 64-bit unsigned atomic max.  Each
        // wave folds its own maximum (no block barrier: a wave leaves as soon
        // as its atomics are issued, and the next block's tile starts sooner)
        unsigned long long wb[D];
#pragma unroll
        for (int d = 0; d < D; ++d) wb[d] = wave_umax64((unsigned long long)__double_as_longlong(wmax[d]));
        if ((tid & 63) == 0) {
            const unsigned blk = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
            unsigned long long* slot = (unsigned long long*)A.wpart + (blk & (A.nslot - 1u)) * D;
#pragma unroll
            for (int d = 0; d < D; ++d) atomicMax(slot + d, wb[d]);
        }
    }
    flush_counters(cnt, A.cnt);
}

template <int N, int D>
__global__ void __launch_bounds__(256) k_relax(double* W, long long nc, EosDev e, unsigned long long* cnt)
{
    constexpr int M = 2 * N + D;
    unsigned c[C_N] = {0, 0, 0, 0, 0, 0, 0};
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < nc; i += (long long)gridDim.x * 256) {
        double w[M];
#pragma unroll
        for (int k = 0; k < M; ++k) w[k] = W[k * nc + i];
        if (relax_cell<N, D>(e, w)) {
#pragma unroll
            for (int k = 0; k < N - 1; ++k) W[(N + D + 1 + k) * nc + i] = w[N + D + 1 + k];
        } else {
            c[C_RELAX_BAD]++;
        }
    }
    flush_counters(c, cnt);
}

// Sec. 3: p*, T* (eq:p_relax, eq:T_relax_e) and the sound speed of the
// four-equation HRM (eq:4_eqn_sos) of every cell; NaN where the state has
// no admissible relaxed state.  Null outputs are skipped.
template <int N, int D>
__global__ void __launch_bounds__(256) k_equilibrium(const double* W, long long nc, EosDev e, double* p_out,
                                                      double* T_out, double* c_out)
{
    constexpr int M = 2 * N + D;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < nc; i += (long long)gridDim.x * 256) {
        double w[M];
#pragma unroll
        for (int k = 0; k < M; ++k) w[k] = W[k * nc + i];
        double p = __builtin_nan(""), T = __builtin_nan(""), c = __builtin_nan("");
        if (relaxed_pT<N, D>(e, w, p, T)) {
            St<N, D> s;
            state_from_W<N, D>(e, w, s);
            hrm4_pc<N, D>(e, s, p, c);
        } else {
            p = T = __builtin_nan("");
        }
        if (p_out) p_out[i] = p;
        if (T_out) T_out[i] = T;
        if (c_out) c_out[i] = c;
    }
}

template <int N, int D>
// only >= 0: the other directions' maxima are 0 (Dirichlet ghost states
// count for the direction normal to their face only)
__global__ void __launch_bounds__(256) k_wavespeed(const double* W, long long nc, EosDev e, int four, int only,
                                                    double* part)
{
    constexpr int M = 2 * N + D;
    __shared__ double sh[4 * 3];
    double m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = 0.0;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < nc; i += (long long)gridDim.x * 256) {
        double w[M];
#pragma unroll
        for (int k = 0; k < M; ++k) w[k] = W[k * nc + i];
        St<N, D> s;
        state_from_W<N, D>(e, w, s);
        double c = s.c;
        if (four) {  // the four-equation model solved directly: its own sound speed
            double p;
            hrm4_pc<N, D>(e, s, p, c);
        }
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (only < 0 || only == d) m[d] = nmax(m[d], fabs(s.u[d]) + c);
    }
    block_max<D>(m, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) part[blockIdx.x * D + d] = m[d];
}

// threads of the one-block reductions of the partials
constexpr int RT = 256;

// this thread's share of the maximum of nb partials (one block of RT
// threads): eight loads in flight per pass instead of one
template <int D>
__device__ inline void partial_max(const double* part, int nb, double* m)
{
    for (int i0 = threadIdx.x; i0 < nb; i0 += RT * 8) {
        double v[8][D];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int d = 0; d < D; ++d) v[u][d] = i0 + RT * u < nb ? part[(i0 + RT * u) * D + d] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int d = 0; d < D; ++d) m[d] = nmax(m[d], v[u][d]);
    }
}

template <int D>
__global__ void __launch_bounds__(RT) k_reduce_max(const double* part, int nb, double* out)
{
    __shared__ double sh[(RT / 64) * 3];
    double m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = 0.0;
    partial_max<D>(part, nb, m);
    block_max<D>(m, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) out[d] = m[d];
}

struct DtArgs {
    int D;
    double dx[3];
    double cfl, dt_fixed, t_end;
};

// Sec. 4.1.2: tau_d = maxs_d / dx_d, dt = CFL / sum tau (or the fixed step),
// lambda_d = dt / (sigma_d dx_d); clipped to t_end with the device time slot[4]
__device__ inline void dt_from_max(const double* maxs, const DtArgs& a, double* slot)
{
    double tau[3] = {0.0, 0.0, 0.0}, ts = 0.0;
    for (int d = 0; d < a.D; ++d) {
        tau[d] = maxs[d] / a.dx[d];
        ts += tau[d];
    }
    double dt = a.dt_fixed > 0.0 ? a.dt_fixed : a.cfl / ts;
    const double t = slot[4];
    if (a.t_end > 0.0 && t + dt > a.t_end) dt = fmax(a.t_end - t, 0.0);
    slot[0] = dt;
    for (int d = 0; d < 3; ++d) slot[1 + d] = d < a.D ? dt / ((tau[d] / ts) * a.dx[d]) : 0.0;
    slot[4] = a.t_end > 0.0 && t + dt >= a.t_end ? a.t_end : t + dt;
}

__global__ void k_dt(const double* maxs, DtArgs a, double* slot)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) dt_from_max(maxs, a, slot);
}

// grid-wide maximum of the wavespeed partials and the time step, one block;
// then the first nclear partials (the slots the last sweep of the step folds
// into) are set to +0, each by the thread that read it
template <int D>
__global__ void __launch_bounds__(RT) k_reduce_dt(double* part, int nb, int nclear, double* maxs, DtArgs a,
                                                   double* slot)
{
    __shared__ double sh[(RT / 64) * 3];
    double m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = 0.0;
    partial_max<D>(part, nb, m);
    for (int i = threadIdx.x; i < nclear; i += RT)
#pragma unroll
        for (int d = 0; d < D; ++d) part[i * D + d] = 0.0;
    block_max<D>(m, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) maxs[d] = m[d];
        dt_from_max(maxs, a, slot);
    }
}

// learned interpolation of n stencils U[i][0..4] (one lane per stencil; the
// whole wave evaluates the network together)
__global__ void __launch_bounds__(64) k_mlp_infer(const MlpPacked* m, const double* U, long long n, double eps,
                                                  double* val, float* om)
{
    const long long i = (long long)blockIdx.x * 64 + threadIdx.x;
    double u[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < n)
#pragma unroll
        for (int j = 0; j < 5; ++j) u[j] = U[i * 5 + j];
    float x[5], z[3], w[3];
    mlp_inputs<double>(u, x);
    mlp_logits(m, x, z);
    const bool ok = mlp_omega(z, x, w);
    if (i < n) {
        val[i] = ok ? mlp_value<double>(u, w) : weno_is<double>(u[0], u[1], u[2], u[3], u[4], eps);
#pragma unroll
        for (int k = 0; k < 3; ++k) om[i * 3 + k] = w[k];
    }
}

__global__ void k_zero_u64(unsigned long long* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

}  // namespace hrm

// ------------------------------------------------------------------ context
struct hrm_ctx {
    int N, D, M;
    int n[3];
    double dx[3];
    int bclo[3], bchi[3];
    int precision, weights, flags;
    long long ncell;
    hrm::EosDev eos;
    hrm::ParDev par;
    double* d_rhs;
    double* d_W1;
    double* d_W2;
    double* d_part;
    int npart;               // wavespeed partial blocks of hrm_max_wavespeed
    int nslot;               // partial slots the last sweep of a step folds its blocks into
    double* d_maxs;
    unsigned long long* d_cnt;
    double* d_bnd[3][2];     // Dirichlet ghost states per face (M x face cells), null elsewhere
    int bnd_set[3][2];
    long long nface[3];      // cells of a face normal to each dimension
    int nbpart[3];           // wavespeed partial blocks per Dirichlet face of that dimension
    hrm::MlpPacked* d_mlp;  // learned weights (HRM_WEIGHTS_MLP)
    int mlp_ready;
    hipStream_t last_stream;
    // hrm_step replay: one captured RK3 step per argument set
    hipStream_t cap_stream;
    hipGraphExec_t gexec;
    double* g_W;
    double* g_slot;
    double g_cfl, g_dt_fixed, g_t_end;
    // opt-in event timing
    int timing_mask;
    int npending;
    int pend_kind[4096];
    hipEvent_t pend_ev[4096][2];
    hipEvent_t pool[4096][2];
    int pool_ready;
    double tms[HRM_NTIMERS];
    long long tcnt[HRM_NTIMERS];
    char err[512];
};

namespace {

int fail(hrm_ctx* c, int code, const char* fmt, const char* a = "", long long v = 0)
{
    if (c) snprintf(c->err, sizeof(c->err), fmt, a, v);
    return code;
}

int check_launch(hrm_ctx* c, const char* what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        snprintf(c->err, sizeof(c->err), "%s: %s", what, hipGetErrorString(e));
        return HRM_EDEVICE;
    }
    return HRM_OK;
}

void fold_timers(hrm_ctx* c)
{
    for (int i = 0; i < c->npending; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->pend_ev[i][0], c->pend_ev[i][1]) == hipSuccess) {
            c->tms[c->pend_kind[i]] += ms;
            c->tcnt[c->pend_kind[i]] += 1;
        }
    }
    c->npending = 0;
}

// records an event pair around the launches in its scope when `kind` is selected
struct TimerScope {
    hrm_ctx* c;
    int kind;
    hipStream_t s;
    int slot;
    TimerScope(hrm_ctx* c_, int kind_, hipStream_t s_) : c(c_), kind(kind_), s(s_), slot(-1)
    {
        if (!c->pool_ready || !((c->timing_mask >> kind) & 1)) return;
        if (c->npending == 4096) {
            (void)hipStreamSynchronize(s);
            fold_timers(c);
        }
        slot = c->npending++;
        c->pend_kind[slot] = kind;
        c->pend_ev[slot][0] = c->pool[slot][0];
        c->pend_ev[slot][1] = c->pool[slot][1];
        (void)hipEventRecord(c->pend_ev[slot][0], s);
    }
    ~TimerScope()
    {
        if (slot >= 0) (void)hipEventRecord(c->pend_ev[slot][1], s);
    }
};

// tile of the sweep in direction dir: BS face threads along it, BA across.
// A tile computes BS faces for BS - 1 cells, so a line of n cells takes
// ceil(n / (BS - 1)) tiles.  Along x (2D, 3D) the 64 x 4 tile gives way to
// 32 x 8 where that needs fewer face threads for the line: a 256-cell line
// takes 5 tiles of 64 (320 face threads, the last tile 4 cells) or 9 of 32
// (288).  Learned weights keep 64 x 4.
void sweep_tile(const hrm_ctx* c, int dir, int& BS, int& BA)
{
    if (c->D == 1) {
        BS = 256;
        BA = 1;
    } else if (dir == 0) {
        const long long n = c->n[0];
        const bool narrow = c->weights != HRM_WEIGHTS_MLP && (n + 30) / 31 * 32 < (n + 62) / 63 * 64 &&
                            (n + 30) / 31 <= 65535;  // tiles along x ride on blockIdx.y
        BS = narrow ? 32 : 64;
        BA = narrow ? 8 : 4;
    } else {
        BS = 16;
        BA = 16;
    }
}

dim3 sweep_grid(const hrm_ctx* c, int dir, int BS, int BA)
{
    const int cells = BS - 1;
    if (dir == 0 && c->D == 1) return dim3((c->n[0] + cells - 1) / cells, (c->n[1] + BA - 1) / BA, c->n[2]);
    if (dir == 0) return dim3((c->n[1] + BA - 1) / BA, (c->n[0] + cells - 1) / cells, c->n[2]);
    if (dir == 1) return dim3((c->n[0] + BA - 1) / BA, (c->n[1] + cells - 1) / cells, c->n[2]);
    return dim3((c->n[0] + BA - 1) / BA, (c->n[2] + cells - 1) / cells, c->n[1]);
}

template <int N, int D>
struct Ops {
    static constexpr int M = 2 * N + D;

    template <int DIR, int BS, int BA>
    static void launch_dir(hrm_ctx* c, hrm::SweepArgs& A, hipStream_t s)
    {
        dim3 blk = DIR == 0 ? dim3(BS, BA) : dim3(BA, BS);
        const dim3 grd = sweep_grid(c, DIR, BS, BA);
        A.bclo = c->bclo[DIR];
        A.bchi = c->bchi[DIR];
        A.blo = c->d_bnd[DIR][0];
        A.bhi = c->d_bnd[DIR][1];
        A.idx = 1.0 / c->dx[DIR];
        TimerScope t(c, HRM_T_SWEEP_X + DIR, s);
        if constexpr (DIR == D - 1) {
            if (A.wpart) {
                launch_kernel<DIR, BS, BA, true>(c, A, grd, blk, s);
                return;
            }
        }
        launch_kernel<DIR, BS, BA, false>(c, A, grd, blk, s);
    }

    template <int DIR, int BS, int BA, bool WS>
    static void launch_kernel(hrm_ctx* c, const hrm::SweepArgs& A, dim3 grd, dim3 blk, hipStream_t s)
    {
        if constexpr (D <= 2 && !(DIR == 0 && BS == 32)) {
            // learned weights: FP64 face arithmetic, one and two dimensions,
            // on the 64 x 4 x-tile (sweep_tile)
            if (c->weights == HRM_WEIGHTS_MLP) {
                hipLaunchKernelGGL((hrm::k_sweep<N, D, DIR, BS, BA, double, 1, WS>), grd, blk, 0, s, A);
                return;
            }
        }
        if (c->precision == HRM_FP32)
            hipLaunchKernelGGL((hrm::k_sweep<N, D, DIR, BS, BA, float, 0, WS>), grd, blk, 0, s, A);
        else
            hipLaunchKernelGGL((hrm::k_sweep<N, D, DIR, BS, BA, double, 0, WS>), grd, blk, 0, s, A);
    }

    // tiles as sweep_tile gives them
    static void sweep(hrm_ctx* c, int dir, hrm::SweepArgs& A, hipStream_t s)
    {
        if constexpr (D == 1) {
            launch_dir<0, 256, 1>(c, A, s);
        } else {
            if (dir == 0) {
                int BS, BA;
                sweep_tile(c, 0, BS, BA);
                if (BS == 32)
                    launch_dir<0, 32, 8>(c, A, s);
                else
                    launch_dir<0, 64, 4>(c, A, s);
            }
            if (dir == 1) launch_dir<1, 16, 16>(c, A, s);
            if constexpr (D >= 3)
                if (dir == 2) launch_dir<2, 16, 16>(c, A, s);
        }
    }

    static void equilibrium(hrm_ctx* c, const double* W, double* p, double* T, double* cs, hipStream_t s)
    {
        const long long nb = std::min<long long>((c->ncell + 255) / 256, 8192);
        hipLaunchKernelGGL((hrm::k_equilibrium<N, D>), dim3((unsigned)nb), dim3(256), 0, s, W, c->ncell, c->eos, p, T,
                           cs);
    }

    static void relax(hrm_ctx* c, double* W, hipStream_t s)
    {
        const long long nb = std::min<long long>((c->ncell + 255) / 256, 8192);
        TimerScope t(c, HRM_T_RELAX, s);
        hipLaunchKernelGGL((hrm::k_relax<N, D>), dim3((unsigned)nb), dim3(256), 0, s, W, c->ncell, c->eos, c->d_cnt);
    }

    // per-block maxima of the cells (ncb blocks), then of the Dirichlet ghost
    // states; returns the number of partial blocks
    static int wavespeed_parts(hrm_ctx* c, const double* W, int ncb, hipStream_t s)
    {
        const int four = (c->flags & HRM_FOUR_EQ) ? 1 : 0;
        hipLaunchKernelGGL((hrm::k_wavespeed<N, D>), dim3(ncb), dim3(256), 0, s, W, c->ncell, c->eos, four, -1,
                           c->d_part);
        int nb = ncb;
        for (int d = 0; d < D; ++d)
            for (int side = 0; side < 2; ++side)
                if (c->d_bnd[d][side]) {
                    hipLaunchKernelGGL((hrm::k_wavespeed<N, D>), dim3(c->nbpart[d]), dim3(256), 0, s,
                                       c->d_bnd[d][side], c->nface[d], c->eos, four, d, c->d_part + (size_t)nb * D);
                    nb += c->nbpart[d];
                }
        return nb;
    }

    // the partials of W in the layout of the final sweep's: nslot slots,
    // then the Dirichlet ghost states
    static void seed_parts(hrm_ctx* c, const double* W, hipStream_t s)
    {
        TimerScope t(c, HRM_T_WAVESPEED, s);
        (void)wavespeed_parts(c, W, c->nslot, s);
    }

    // the time step from the partials of seed_parts or of the last final sweep
    static void reduce_dt(hrm_ctx* c, const hrm::DtArgs& a, double* slot, hipStream_t s)
    {
        TimerScope t(c, HRM_T_WAVESPEED, s);
        int nb = c->nslot;
        for (int d = 0; d < D; ++d)
            for (int side = 0; side < 2; ++side)
                if (c->d_bnd[d][side]) nb += c->nbpart[d];
        hipLaunchKernelGGL((hrm::k_reduce_dt<D>), dim3(1), dim3(hrm::RT), 0, s, c->d_part, nb, c->nslot, c->d_maxs, a,
                           slot);
    }

    static void wavespeed(hrm_ctx* c, const double* W, double* out, hipStream_t s)
    {
        TimerScope t(c, HRM_T_WAVESPEED, s);
        const int nb = wavespeed_parts(c, W, c->npart, s);
        hipLaunchKernelGGL((hrm::k_reduce_max<D>), dim3(1), dim3(hrm::RT), 0, s, c->d_part, nb, out);
    }
};

template <typename Fn>
int dispatch(hrm_ctx* c, Fn&& fn)
{
    switch (c->N * 10 + c->D) {
    case 21: fn(Ops<2, 1>()); return HRM_OK;
    case 22: fn(Ops<2, 2>()); return HRM_OK;
    case 23: fn(Ops<2, 3>()); return HRM_OK;
    case 31: fn(Ops<3, 1>()); return HRM_OK;
    case 32: fn(Ops<3, 2>()); return HRM_OK;
    case 33: fn(Ops<3, 3>()); return HRM_OK;
    default: return fail(c, HRM_EUNSUPPORTED, "N=%s%lld with this dim is not built", "", c->N);
    }
}

hrm::SweepArgs base_args(hrm_ctx* c)
{
    hrm::SweepArgs A;
    memset(&A, 0, sizeof(A));
    A.cnt = c->d_cnt;
    A.ncell = c->ncell;
    for (int d = 0; d < 3; ++d) A.n[d] = c->n[d];
    A.e = c->eos;
    A.P = c->par;
    return A;
}

int check_boundary(hrm_ctx* c);

// all directions of L(W_s); with `stage` the last one applies the stage
// update (and writes the wavespeed partials of its output into wpart)
int run_operator(hrm_ctx* c, const double* Ws, const double* Wn, double* Wout, double* rhs, const double* slot,
                 bool stage, double a, double b, int relax, hipStream_t s, double* wpart = nullptr, int hold = 0)
{
    if (c->weights == HRM_WEIGHTS_MLP && !c->mlp_ready)
        return fail(c, HRM_EINVAL, "learned weights selected but hrm_set_mlp not called%s");
    if (const int rb = check_boundary(c)) return rb;
    hrm::SweepArgs A = base_args(c);
    A.Ws = Ws;
    A.Wn = Wn;
    A.Wout = Wout;
    A.rhs = rhs;
    A.slot = slot;
    A.a = a;
    A.b = b;
    A.relax = relax;
    A.hold = hold;
    A.wpart = stage ? wpart : nullptr;
    A.nslot = (unsigned)c->nslot;
    int rc = HRM_OK;
    for (int d = 0; d < c->D; ++d) {
        const bool last = d == c->D - 1;
        A.mode = (stage && last) ? hrm::MODE_FINAL : (d == 0 ? hrm::MODE_WRITE : hrm::MODE_ADD);
        rc = dispatch(c, [&](auto ops) { decltype(ops)::sweep(c, d, A, s); });
        if (rc != HRM_OK) return rc;
        if ((rc = check_launch(c, "sweep")) != HRM_OK) return rc;
    }
    return rc;
}

bool valid_ptr(const void* p) { return p != nullptr; }

// every Dirichlet face has had its state set
int check_boundary(hrm_ctx* c)
{
    for (int d = 0; d < c->D; ++d)
        for (int side = 0; side < 2; ++side)
            if (c->d_bnd[d][side] && !c->bnd_set[d][side])
                return fail(c, HRM_EINVAL, "Dirichlet state of dimension %s%lld not set (hrm_set_boundary_state)", "",
                            d);
    return HRM_OK;
}

hrm::DtArgs dt_args(hrm_ctx* c, double cfl, double dt_fixed, double t_end)
{
    hrm::DtArgs a;
    a.D = c->D;
    for (int d = 0; d < 3; ++d) a.dx[d] = c->dx[d];
    a.cfl = cfl;
    a.dt_fixed = dt_fixed;
    a.t_end = t_end;
    return a;
}

// the wavespeed partials of W^n for the first step of a run (the later
// steps find them written by the final sweep of the step before)
int seed_enqueue(hrm_ctx* c, const double* d_W, hipStream_t s)
{
    int rc = check_boundary(c);
    if (rc == HRM_OK) rc = dispatch(c, [&](auto ops) { decltype(ops)::seed_parts(c, d_W, s); });
    if (rc == HRM_OK) rc = check_launch(c, "hrm_advance wavespeed");
    return rc;
}

// the launches of one RK3 step on stream s: time step from the partials,
// three stages with the relaxation, the last one leaving the partials of
// W^{n+1}
int step_enqueue(hrm_ctx* c, double* d_W, double cfl, double dt_fixed, double t_end, double* d_slot, hipStream_t s)
{
    static const double RK_A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    static const double RK_B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    const hrm::DtArgs a = dt_args(c, cfl, dt_fixed, t_end);
    int rc = check_boundary(c);
    if (rc == HRM_OK) rc = dispatch(c, [&](auto ops) { decltype(ops)::reduce_dt(c, a, d_slot, s); });
    if (rc == HRM_OK) rc = check_launch(c, "hrm_advance time step");
    if (rc == HRM_OK)
        rc = run_operator(c, d_W, d_W, c->d_W1, c->d_rhs, d_slot, true, RK_A[0], RK_B[0], 1, s, nullptr, 1);
    if (rc == HRM_OK)
        rc = run_operator(c, c->d_W1, d_W, c->d_W2, c->d_rhs, d_slot, true, RK_A[1], RK_B[1], 1, s, nullptr, 1);
    if (rc == HRM_OK)
        rc = run_operator(c, c->d_W2, d_W, d_W, c->d_rhs, d_slot, true, RK_A[2], RK_B[2], 1, s, c->d_part, 1);
    return rc;
}

void drop_graph(hrm_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
}

}  // namespace

extern "C" {

void hrm_default_params(hrm_params* p)
{
    if (!p) return;
    p->eps_weno = 1e-15;
    p->eps_i_ar = 1e-10;
    p->eps_i_a = 1e-10;
    p->hs_i_ar = 1e-11;
    p->hs_i_a = 1e-11;
    p->hs_i_rc2 = 1e-9;
    p->eps_f_ar = 1e-10;
    p->eps_f_a = 1e-10;
    p->eps_f_re = 1e-8;
    p->hs_f_ar = 1e-11;
    p->hs_f_a = 1e-11;
    p->hs_f_re = 1e-9;
    p->Cs = 1e12;
    p->qexp = 2.0;
    p->psi = 256.0 / 175.0;
}

const char* hrm_last_error(const hrm_ctx* ctx) { return ctx ? ctx->err : "NULL context"; }

int hrm_create(const hrm_grid* g, const hrm_eos* e, const hrm_params* prm, hrm_ctx** out)
{
    if (!out) return HRM_EINVAL;
    *out = nullptr;
    if (!g || !e) return HRM_EINVAL;
    if (g->dim < 1 || g->dim > 3) return HRM_EINVAL;
    if (e->nspecies < 2 || e->nspecies > HRM_MAX_SPECIES) return HRM_EINVAL;
    for (int d = 0; d < 3; ++d) {
        if (g->n[d] < 1 || (d >= g->dim && g->n[d] != 1)) return HRM_EINVAL;
        if (d < g->dim && !(g->dx[d] > 0.0)) return HRM_EINVAL;
        if (d < g->dim) {
            for (int side = 0; side < 2; ++side) {
                const int bc = side ? g->bc_hi[d] : g->bc_lo[d];
                if (bc != HRM_BC_TRANSMISSIVE && bc != HRM_BC_PERIODIC && bc != HRM_BC_DIRICHLET) return HRM_EINVAL;
            }
            if ((g->bc_lo[d] == HRM_BC_PERIODIC) != (g->bc_hi[d] == HRM_BC_PERIODIC)) return HRM_EINVAL;
        }
    }
    for (int k = 0; k < e->nspecies; ++k) {
        if (!(e->gamma[k] > 1.0) || !(e->cv[k] > 0.0) || !(e->pinf[k] >= 0.0)) return HRM_EINVAL;
        if (k > 0 && e->pinf[k] != 0.0) return HRM_EINVAL;  // one stiffened gas, species 0 (Sec. 4.2)
    }
    if (g->precision != HRM_FP64 && g->precision != HRM_FP32) return HRM_EINVAL;
    if (g->weights != HRM_WEIGHTS_IS && g->weights != HRM_WEIGHTS_MLP) return HRM_EINVAL;
    if (g->weights == HRM_WEIGHTS_MLP && (g->precision != HRM_FP64 || g->dim > 2)) return HRM_EUNSUPPORTED;

    hrm_ctx* c = new (std::nothrow) hrm_ctx;
    if (!c) return HRM_ENOMEM;
    memset(c, 0, sizeof(*c));
    c->N = e->nspecies;
    c->D = g->dim;
    c->M = 2 * c->N + c->D;
    for (int d = 0; d < 3; ++d) {
        c->n[d] = g->n[d];
        c->dx[d] = d < g->dim ? g->dx[d] : 1.0;
        c->bclo[d] = d < g->dim ? g->bc_lo[d] : HRM_BC_TRANSMISSIVE;
        c->bchi[d] = d < g->dim ? g->bc_hi[d] : HRM_BC_TRANSMISSIVE;
    }
    c->precision = g->precision;
    c->weights = g->weights;
    c->flags = g->flags;
    c->ncell = (long long)g->n[0] * g->n[1] * g->n[2];
    if (!((c->N == 2 || c->N == 3))) {
        delete c;
        return HRM_EUNSUPPORTED;
    }
    for (int d = 0; d < c->D; ++d) {
        // every sweep launch within the grid limits (y and z at most 65535 blocks)
        int BS, BA;
        sweep_tile(c, d, BS, BA);
        const dim3 gd = sweep_grid(c, d, BS, BA);
        if (gd.y > 65535u || gd.z > 65535u) {
            delete c;
            return HRM_EUNSUPPORTED;
        }
    }
    for (int k = 0; k < hrm::MAXN; ++k) {
        const bool on = k < c->N;
        c->eos.g[k] = on ? e->gamma[k] : 2.0;
        c->eos.cv[k] = on ? e->cv[k] : 1.0;
        c->eos.pinf[k] = on ? e->pinf[k] : 0.0;
        c->eos.q[k] = on ? e->q[k] : 0.0;
        c->eos.ig1[k] = 1.0 / (c->eos.g[k] - 1.0);
        c->eos.gpi1[k] = c->eos.g[k] * c->eos.pinf[k] / (c->eos.g[k] - 1.0);
        c->eos.cp[k] = c->eos.g[k] * c->eos.cv[k];
    }
    hrm_params p;
    if (prm)
        p = *prm;
    else
        hrm_default_params(&p);
    hrm::ParDev& P = c->par;
    P.eps_weno = p.eps_weno;
    P.eps_i_ar = p.eps_i_ar;
    P.eps_i_a = p.eps_i_a;
    P.hs_i_ar = p.hs_i_ar;
    P.hs_i_a = p.hs_i_a;
    P.hs_i_rc2 = p.hs_i_rc2;
    P.eps_f_ar = p.eps_f_ar;
    P.eps_f_a = p.eps_f_a;
    P.eps_f_re = p.eps_f_re;
    P.hs_f_ar = p.hs_f_ar;
    P.hs_f_a = p.hs_f_a;
    P.hs_f_re = p.hs_f_re;
    P.Cs = p.Cs;
    P.qexp = p.qexp;
    P.psi = p.psi;
    P.hcs_a = 75.0 * p.psi / 128.0 - 37.0 / 60.0;
    P.hcs_b = 25.0 * p.psi / 256.0 - 2.0 / 15.0;
    P.hcs_c = 3.0 * p.psi / 256.0 - 1.0 / 60.0;
    P.flags = g->flags;
    if (g->flags & HRM_FOUR_EQ) P.flags |= HRM_FIRST_ORDER;  // the direct HRM solver is first order
    P.fast_flux_limiter = p.eps_f_ar >= p.hs_f_ar && p.eps_f_a >= p.hs_f_a && p.eps_f_re >= p.hs_f_re;

    const size_t bytes = sizeof(double) * (size_t)c->M * (size_t)c->ncell;
    c->npart = (int)std::min<long long>((c->ncell + 255) / 256, 2048);
    {
        int BS, BA;
        sweep_tile(c, c->D - 1, BS, BA);
        const dim3 g = sweep_grid(c, c->D - 1, BS, BA);
        // the largest power of two up to the block count and 2048, so that
        // every slot receives at least one block
        const long long nblk = (long long)g.x * g.y * g.z;
        c->nslot = 1;
        while (c->nslot < 2048 && 2ll * c->nslot <= nblk) c->nslot *= 2;
    }
    int nparts = std::max(c->npart, c->nslot);
    for (int d = 0; d < 3; ++d) {
        c->nface[d] = c->ncell / c->n[d];
        c->nbpart[d] = (int)std::min<long long>((c->nface[d] + 255) / 256, 256);
        if (d < c->D)
            for (int side = 0; side < 2; ++side)
                if ((side ? c->bchi[d] : c->bclo[d]) == HRM_BC_DIRICHLET) nparts += c->nbpart[d];
    }
    bool ok = true;
    for (int d = 0; d < c->D; ++d)
        for (int side = 0; side < 2; ++side)
            if ((side ? c->bchi[d] : c->bclo[d]) == HRM_BC_DIRICHLET)
                ok = ok && hipMalloc((void**)&c->d_bnd[d][side], sizeof(double) * (size_t)c->M * c->nface[d]) ==
                               hipSuccess;
    if (c->D > 1) ok = ok && hipMalloc((void**)&c->d_rhs, bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->d_W1, bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->d_W2, bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->d_part, sizeof(double) * 3 * (size_t)nparts) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->d_maxs, sizeof(double) * 4) == hipSuccess;
    ok = ok && hipMalloc((void**)&c->d_cnt, sizeof(unsigned long long) * 8) == hipSuccess;
    if (c->weights == HRM_WEIGHTS_MLP) ok = ok && hipMalloc((void**)&c->d_mlp, sizeof(hrm::MlpPacked)) == hipSuccess;
    P.mlp = c->d_mlp;
    if (ok) ok = hipMemset(c->d_cnt, 0, sizeof(unsigned long long) * 8) == hipSuccess;
    if (ok) ok = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        hrm_destroy(c);
        return HRM_ENOMEM;
    }
    *out = c;
    return HRM_OK;
}

int hrm_destroy(hrm_ctx* c)
{
    if (!c) return HRM_EINVAL;
    (void)hipDeviceSynchronize();
    if (c->pool_ready)
        for (int i = 0; i < 4096; ++i) {
            (void)hipEventDestroy(c->pool[i][0]);
            (void)hipEventDestroy(c->pool[i][1]);
        }
    for (int d = 0; d < 3; ++d)
        for (int side = 0; side < 2; ++side) (void)hipFree(c->d_bnd[d][side]);
    (void)hipFree(c->d_rhs);
    (void)hipFree(c->d_W1);
    (void)hipFree(c->d_W2);
    (void)hipFree(c->d_part);
    (void)hipFree(c->d_maxs);
    (void)hipFree(c->d_cnt);
    (void)hipFree(c->d_mlp);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return HRM_OK;
}

int hrm_max_wavespeed(hrm_ctx* c, const double* d_W, double* d_out, void* stream)
{
    if (!c) return HRM_EINVAL;
    if (!valid_ptr(d_W) || !valid_ptr(d_out)) return fail(c, HRM_EINVAL, "hrm_max_wavespeed: NULL pointer%s", "");
    if (const int rb = check_boundary(c)) return rb;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    const int rc = dispatch(c, [&](auto ops) { decltype(ops)::wavespeed(c, d_W, d_out, s); });
    return rc != HRM_OK ? rc : check_launch(c, "hrm_max_wavespeed");
}

int hrm_compute_dt(hrm_ctx* c, const double* d_maxspeed, double cfl, double dt_fixed, double t_end, double* d_slot,
                   void* stream)
{
    if (!c) return HRM_EINVAL;
    if (!valid_ptr(d_maxspeed) || !valid_ptr(d_slot)) return fail(c, HRM_EINVAL, "hrm_compute_dt: NULL pointer%s");
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(c, HRM_EINVAL, "hrm_compute_dt: need cfl > 0 or dt_fixed > 0%s");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    TimerScope t(c, HRM_T_DT, s);
    hipLaunchKernelGGL(hrm::k_dt, dim3(1), dim3(64), 0, s, d_maxspeed, dt_args(c, cfl, dt_fixed, t_end), d_slot);
    return check_launch(c, "hrm_compute_dt");
}

int hrm_rhs(hrm_ctx* c, const double* d_W, double* d_L, const double* d_slot, void* stream)
{
    if (!c) return HRM_EINVAL;
    if (!valid_ptr(d_W) || !valid_ptr(d_L) || !valid_ptr(d_slot)) return fail(c, HRM_EINVAL, "hrm_rhs: NULL pointer%s");
    if ((const double*)d_L == d_W) return fail(c, HRM_EINVAL, "hrm_rhs: d_L aliases d_W%s");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    return run_operator(c, d_W, nullptr, nullptr, d_L, d_slot, false, 0.0, 0.0, 0, s);
}

int hrm_rk_stage(hrm_ctx* c, int stage, const double* d_Wn, const double* d_Ws, double* d_Wout, const double* d_slot,
                 void* stream)
{
    static const double RK_A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
    static const double RK_B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
    if (!c) return HRM_EINVAL;
    if (stage < 0 || stage > 2) return fail(c, HRM_EINVAL, "hrm_rk_stage: stage %s%lld not in 0..2", "", stage);
    if (!valid_ptr(d_Wn) || !valid_ptr(d_Ws) || !valid_ptr(d_Wout) || !valid_ptr(d_slot))
        return fail(c, HRM_EINVAL, "hrm_rk_stage: NULL pointer%s");
    if ((const double*)d_Wout == d_Ws) return fail(c, HRM_EINVAL, "hrm_rk_stage: d_Wout aliases d_Ws%s");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    return run_operator(c, d_Ws, d_Wn, d_Wout, c->d_rhs, d_slot, true, RK_A[stage], RK_B[stage],
                        (c->flags & HRM_FUSE_RELAX) ? 1 : 0, s);
}

int hrm_set_boundary_state(hrm_ctx* c, int dim, int side, const double* d_state, void* stream)
{
    if (!c) return HRM_EINVAL;
    if (dim < 0 || dim >= c->D || side < 0 || side > 1 || !c->d_bnd[dim][side])
        return fail(c, HRM_EINVAL, "hrm_set_boundary_state: face (dim %s%lld) is not a Dirichlet face", "", dim);
    if (!valid_ptr(d_state)) return fail(c, HRM_EINVAL, "hrm_set_boundary_state: NULL pointer%s");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (hipMemcpyAsync(c->d_bnd[dim][side], d_state, sizeof(double) * (size_t)c->M * c->nface[dim],
                       hipMemcpyDeviceToDevice, s) != hipSuccess)
        return fail(c, HRM_EDEVICE, "hrm_set_boundary_state: copy failed: %s", hipGetErrorString(hipGetLastError()));
    c->bnd_set[dim][side] = 1;
    return HRM_OK;
}

int hrm_relax(hrm_ctx* c, double* d_W, void* stream)
{
    if (!c) return HRM_EINVAL;
    if (!valid_ptr(d_W)) return fail(c, HRM_EINVAL, "hrm_relax: NULL pointer%s");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    const int rc = dispatch(c, [&](auto ops) { decltype(ops)::relax(c, d_W, s); });
    return rc != HRM_OK ? rc : check_launch(c, "hrm_relax");
}

int hrm_equilibrium_state(hrm_ctx* c, const double* d_W, double* d_p, double* d_T, double* d_c, void* stream)
{
    if (!c) return HRM_EINVAL;
    if (!valid_ptr(d_W)) return fail(c, HRM_EINVAL, "hrm_equilibrium_state: NULL state%s");
    if (!d_p && !d_T && !d_c) return HRM_OK;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    const int rc = dispatch(c, [&](auto ops) { decltype(ops)::equilibrium(c, d_W, d_p, d_T, d_c, s); });
    return rc != HRM_OK ? rc : check_launch(c, "hrm_equilibrium_state");
}

int hrm_set_mlp(hrm_ctx* c, const float* h_params)
{
    if (!c) return HRM_EINVAL;
    if (c->weights != HRM_WEIGHTS_MLP) return fail(c, HRM_EINVAL, "hrm_set_mlp: the grid uses App. C weights%s");
    if (!h_params) return fail(c, HRM_EINVAL, "hrm_set_mlp: NULL parameters%s");
    hrm::MlpPacked pk;
    hrm::mlp_pack_host(h_params, &pk);
    // ordered after the work already enqueued by this context
    if (hipStreamSynchronize(c->last_stream) != hipSuccess ||
        hipMemcpy(c->d_mlp, &pk, sizeof(pk), hipMemcpyHostToDevice) != hipSuccess)
        return fail(c, HRM_EDEVICE, "hrm_set_mlp: copy failed%s");
    c->mlp_ready = 1;
    return HRM_OK;
}

int hrm_mlp_infer(hrm_ctx* c, const double* d_U5, long long n, double* d_val, float* d_omega, void* stream)
{
    if (!c) return HRM_EINVAL;
    if (c->weights != HRM_WEIGHTS_MLP || !c->mlp_ready)
        return fail(c, HRM_EINVAL, "hrm_mlp_infer: no learned weights on this grid%s");
    if (n < 0 || (n > 0 && (!valid_ptr(d_U5) || !valid_ptr(d_val) || !d_omega)))
        return fail(c, HRM_EINVAL, "hrm_mlp_infer: bad arguments%s");
    if (n == 0) return HRM_OK;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    hipLaunchKernelGGL(hrm::k_mlp_infer, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, c->d_mlp, d_U5, n,
                       c->par.eps_weno, d_val, d_omega);
    return check_launch(c, "hrm_mlp_infer");
}

int hrm_advance(hrm_ctx* c, double* d_W, int nsteps, double cfl, double dt_fixed, double t_end, double* d_slot,
                void* stream)
{
    if (!c) return HRM_EINVAL;
    if (!valid_ptr(d_W) || !valid_ptr(d_slot)) return fail(c, HRM_EINVAL, "hrm_advance: NULL pointer%s");
    if (nsteps < 0) return fail(c, HRM_EINVAL, "hrm_advance: nsteps = %s%lld < 0", "", nsteps);
    if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return fail(c, HRM_EINVAL, "hrm_advance: need cfl > 0 or dt_fixed > 0%s");
    if (c->weights == HRM_WEIGHTS_MLP && !c->mlp_ready)
        return fail(c, HRM_EINVAL, "learned weights selected but hrm_set_mlp not called%s");
    if (nsteps == 0) return HRM_OK;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    int rc = seed_enqueue(c, d_W, s);
    if (rc != HRM_OK) return rc;
    if ((c->flags & HRM_NO_GRAPH) || c->timing_mask) {
        for (int k = 0; k < nsteps && rc == HRM_OK; ++k) rc = step_enqueue(c, d_W, cfl, dt_fixed, t_end, d_slot, s);
        return rc;
    }
    const bool same = c->gexec && c->g_W == d_W && c->g_slot == d_slot && c->g_cfl == cfl &&
                      c->g_dt_fixed == dt_fixed && c->g_t_end == t_end;
    if (!same) {
        drop_graph(c);
        if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
            return fail(c, HRM_EDEVICE, "hrm_advance: stream capture failed%s");
        rc = step_enqueue(c, d_W, cfl, dt_fixed, t_end, d_slot, c->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
        if (rc != HRM_OK || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return rc != HRM_OK ? rc : fail(c, HRM_EDEVICE, "hrm_advance: end capture: %s", hipGetErrorString(ec));
        }
        const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            c->gexec = nullptr;
            return fail(c, HRM_EDEVICE, "hrm_advance: graph instantiate: %s", hipGetErrorString(ei));
        }
        c->g_W = d_W;
        c->g_slot = d_slot;
        c->g_cfl = cfl;
        c->g_dt_fixed = dt_fixed;
        c->g_t_end = t_end;
    }
    for (int k = 0; k < nsteps; ++k)
        if (hipGraphLaunch(c->gexec, s) != hipSuccess)
            return fail(c, HRM_EDEVICE, "hrm_advance: graph launch: %s", hipGetErrorString(hipGetLastError()));
    return HRM_OK;
}

int hrm_step(hrm_ctx* c, double* d_W, double cfl, double dt_fixed, double t_end, double* d_slot, void* stream)
{
    return hrm_advance(c, d_W, 1, cfl, dt_fixed, t_end, d_slot, stream);
}

int hrm_get_diagnostics(hrm_ctx* c, hrm_diag* out)
{
    if (!c || !out) return HRM_EINVAL;
    if (hipStreamSynchronize(c->last_stream) != hipSuccess ||
        hipMemcpy(out, c->d_cnt, sizeof(hrm_diag), hipMemcpyDeviceToHost) != hipSuccess) {
        snprintf(c->err, sizeof(c->err), "hrm_get_diagnostics: %s", hipGetErrorString(hipGetLastError()));
        return HRM_EDEVICE;
    }
    return out->relax_bad ? HRM_EADMISSIBLE : HRM_OK;
}

int hrm_reset_diagnostics(hrm_ctx* c, void* stream)
{
    if (!c) return HRM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    hipLaunchKernelGGL(hrm::k_zero_u64, dim3(1), dim3(64), 0, s, c->d_cnt, 8);
    return check_launch(c, "hrm_reset_diagnostics");
}

int hrm_set_timing(hrm_ctx* c, int mask)
{
    if (!c) return HRM_EINVAL;
    if (mask && !c->pool_ready) {
        for (int i = 0; i < 4096; ++i)
            if (hipEventCreate(&c->pool[i][0]) != hipSuccess || hipEventCreate(&c->pool[i][1]) != hipSuccess) {
                snprintf(c->err, sizeof(c->err), "hrm_set_timing: %s", hipGetErrorString(hipGetLastError()));
                return HRM_EDEVICE;
            }
        c->pool_ready = 1;
    }
    c->timing_mask = mask;
    return HRM_OK;
}

int hrm_get_timing(hrm_ctx* c, double* ms, long long* counts)
{
    if (!c || !ms || !counts) return HRM_EINVAL;
    if (hipStreamSynchronize(c->last_stream) != hipSuccess) {
        snprintf(c->err, sizeof(c->err), "hrm_get_timing: %s", hipGetErrorString(hipGetLastError()));
        return HRM_EDEVICE;
    }
    fold_timers(c);
    for (int k = 0; k < HRM_NTIMERS; ++k) {
        ms[k] = c->tms[k];
        counts[k] = c->tcnt[k];
        c->tms[k] = 0.0;
        c->tcnt[k] = 0;
    }
    return HRM_OK;
}

}  // extern "C"
