// hrm_batch.hip -- ragged ensemble of independent 1D problems in one
// persistent launch (gfx950).  Declarations and semantics: include/hrm.h.
//
// Each workgroup takes problem ids from an atomic queue (problems sorted
// longest first on the host) and advances its problem by K SSP-RK3 steps of
// the fractional algorithm: per-problem wavespeed and dt (Sec. 4.1.2), then
// three stages, each a loop over LDS tiles of the problem (same face
// arithmetic as k_sweep) with the Shu-Osher update and the relaxation fused
// (Sec. 4.4, Sec. 4.2).  A launch processes every problem once; hrm_batch_run
// replays a captured graph of (queue reset, persistent launch) pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "hrm.h"
#include "hrm_face.hpp"

namespace hrm {

struct BatchArgs {
    double* W;   // state (M x T), in/out
    double* W1;  // stage buffers (M x T)
    double* W2;
    const long long* off;  // problem b owns cells off[b] .. off[b+1]-1
    const double* dx;
    const int* order;      // processing order (longest first)
    double* t;             // per-problem time
    const double* tend;    // per-problem end time (<= 0: none)
    int* queue;
    unsigned long long* cnt;
    long long T;
    int nprob;
    int ksteps;
    double cfl;
    EosDev e;
    ParDev P;
};

__global__ void k_set_int(int* p, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// a workgroup-uniform double (read from LDS) moved to scalar registers
__device__ inline double uniform(double v)
{
    const unsigned long long u = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int N, int BS, typename R>
__global__ void __launch_bounds__(BS, 3) k_batch(const BatchArgs A)
{
    constexpr int D = 1;
    using F = NodeFields<N, D>;
    constexpr int M = 2 * N + D, IA = N + D + 1;
    constexpr int NA = N > 1 ? N - 1 : 1;
    constexpr int LN = BS + 5;
    constexpr int FS = LN;
    static_assert(BS % 64 == 0 && BS <= 256, "block size");
    __shared__ double lds[F::COUNT * FS];
    __shared__ double sh[12];
    __shared__ double sdt[3];
    __shared__ int spid;
    const int ts = threadIdx.x;
    const long long T = A.T;
    unsigned cnt[C_N] = {0, 0, 0, 0, 0, 0, 0};

    for (;;) {
        if (ts == 0) spid = atomicAdd(A.queue, 1);
        __syncthreads();
        const int pid = __builtin_amdgcn_readfirstlane(spid);
        __syncthreads();
        if (pid >= A.nprob) break;
        const int b = A.order[pid];
        const long long base = A.off[b];
        const int n = (int)(A.off[b + 1] - base);
        const double dxb = A.dx[b];
        const double idx = 1.0 / dxb;

        for (int step = 0; step < A.ksteps; ++step) {
            // per-problem wavespeed and time step (1D: sigma = 1, lambda = dt/dx)
            double m[1] = {0.0};
            for (int i = ts; i < n; i += BS) {
                double w[M];
#pragma unroll
                for (int c = 0; c < M; ++c) w[c] = A.W[c * T + base + i];
                St<N, D> s;
                state_from_W<N, D>(A.e, w, s);
                m[0] = nmax(m[0], fabs(s.u[0]) + s.c);
            }
            block_max<1>(m, sh);
            if (ts == 0) {
                // the step is clipped so that t does not pass the problem's
                // end time (as hrm_compute_dt does); a problem that has
                // reached it takes no further steps
                const double tau = m[0] / dxb;
                const double t = A.t[b], te = A.tend[b];
                double dt = A.cfl / tau;
                if (te > 0.0 && t + dt > te) dt = fmax(te - t, 0.0);
                sdt[0] = dt;
                sdt[1] = dt / ((tau / tau) * dxb);
                sdt[2] = te > 0.0 && t >= te ? 1.0 : 0.0;
                if (sdt[2] == 0.0) A.t[b] = te > 0.0 && t + dt >= te ? te : t + dt;
            }
            __syncthreads();
            const double dt = uniform(sdt[0]), lam = uniform(sdt[1]);
            if (uniform(sdt[2]) != 0.0) break;

            for (int stage = 0; stage < 3; ++stage) {
                const double* Ws = stage == 0 ? A.W : (stage == 1 ? A.W1 : A.W2);
                double* Wout = stage == 0 ? A.W1 : (stage == 1 ? A.W2 : A.W);
                // Shu-Osher coefficients (a, b) of the three stages
                const double ca = stage == 0 ? 0.0 : (stage == 1 ? 3.0 / 4.0 : 1.0 / 3.0);
                const double cb = stage == 0 ? 1.0 : (stage == 1 ? 1.0 / 4.0 : 2.0 / 3.0);
                for (int c0 = 0; c0 < n; c0 += BS - 1) {
                    const EosDev& e = A.e;
                    const ParDev& P = A.P;
                    // stage the tile c0-3 .. c0+BS+1 with its primitives
                    // (at raised priority, as in k_sweep)
                    __builtin_amdgcn_s_setprio(3);
                    for (int l = ts; l < LN; l += BS) {
                        const int g = map_bc(c0 - 3 + l, n, HRM_BC_TRANSMISSIVE, HRM_BC_TRANSMISSIVE);
                        double W[M];
#pragma unroll
                        for (int c = 0; c < M; ++c) W[c] = Ws[c * T + base + g];
                        St<N, D> s;
                        state_from_W<N, D>(e, W, s);
#pragma unroll
                        for (int c = 0; c < M; ++c) lds[c * FS + l] = W[c];
                        lds[F::U * FS + l] = s.u[0];
                        lds[F::P * FS + l] = s.p;
                        lds[F::RHO * FS + l] = s.rho;
                        lds[F::C * FS + l] = s.c;
                        lds[F::RC2 * FS + l] = s.rc2;
                    }
                    __builtin_amdgcn_s_setprio(0);
                    __syncthreads();
                    double G[M], Gp[NA];
                    // a wave whose faces all lie beyond face n (the last tile of
                    // a problem) skips them and leaves their slots, which no
                    // cell reads, unwritten
                    const bool live = c0 + (ts & ~63) <= n;
                    if (live) {
                        unsigned lc = 0;  // packed counts of this face (cnt_one)
                        face_flux<N, D, 0, 1, FS, R, 0, false>(lds + ts, e, P, lam, G, Gp, lc);
                        const int f = c0 + ts;  // counted once, as in k_sweep
                        if (f <= n && (ts < BS - 1 || f == n))
#pragma unroll
                            for (int k = 0; k < C_N; ++k) cnt[k] += cnt_get(lc, k);
                    }
                    __syncthreads();
                    if (live) {
#pragma unroll
                        for (int c = 0; c < M; ++c) lds[c * FS + ts] = G[c];
#pragma unroll
                        for (int k = 0; k < N - 1; ++k) lds[(M + k) * FS + ts] = Gp[k];
                    }
                    __syncthreads();
                    const int ci = c0 + ts;
                    if (ts < BS - 1 && ci < n) {
                        const long long cell = base + ci;
                        double w[M];
#pragma unroll
                        for (int c = 0; c < M; ++c) {
                            const double gp = c >= IA ? lds[(M + c - IA) * FS + ts] : lds[c * FS + ts];
                            const double L = -(lds[c * FS + ts + 1] - gp) * idx;
                            w[c] = ca * A.W[c * T + cell] + cb * (Ws[c * T + cell] + dt * L);
                        }
                        if (!relax_cell<N, D>(e, w)) cnt[C_RELAX_BAD]++;
#pragma unroll
                        for (int c = 0; c < M; ++c) Wout[c * T + cell] = w[c];
                    }
                    __syncthreads();
                }
            }
        }
    }
    flush_counters(cnt, A.cnt);
}

}  // namespace hrm

struct hrm_batch {
    int N, M, nprob, precision, flags;
    long long T;
    hrm::EosDev eos;
    hrm::ParDev par;
    double* d_W1;
    double* d_W2;
    long long* d_off;
    double* d_dx;
    int* d_order;
    double* d_t;
    double* d_tend;
    int* d_queue;
    unsigned long long* d_cnt;
    int threads, blocks, ksteps;
    hipStream_t cap_stream;
    hipGraphExec_t gexec;
    double* g_W;
    double g_cfl;
    hipStream_t last_stream;
    char err[512];
};

namespace {

int bfail(hrm_batch* b, int code, const char* msg)
{
    if (b) snprintf(b->err, sizeof(b->err), "%s", msg);
    return code;
}

template <int N, int BS>
void launch_bs(hrm_batch* b, const hrm::BatchArgs& A, hipStream_t s)
{
    if (b->precision == HRM_FP32)
        hipLaunchKernelGGL((hrm::k_batch<N, BS, float>), dim3(b->blocks), dim3(BS), 0, s, A);
    else
        hipLaunchKernelGGL((hrm::k_batch<N, BS, double>), dim3(b->blocks), dim3(BS), 0, s, A);
}

template <int N>
int launch_n(hrm_batch* b, const hrm::BatchArgs& A, hipStream_t s)
{
    switch (b->threads) {
    case 64: launch_bs<N, 64>(b, A, s); return HRM_OK;
    case 128: launch_bs<N, 128>(b, A, s); return HRM_OK;
    case 256: launch_bs<N, 256>(b, A, s); return HRM_OK;
    default: return bfail(b, HRM_EINVAL, "hrm_batch: threads must be 64, 128 or 256");
    }
}

// one chunk: reset the queue, then the persistent launch advancing every problem K steps
int enqueue_chunk(hrm_batch* b, double* d_W, double cfl, hipStream_t s)
{
    hrm::BatchArgs A;
    memset(&A, 0, sizeof(A));
    A.W = d_W;
    A.W1 = b->d_W1;
    A.W2 = b->d_W2;
    A.off = b->d_off;
    A.dx = b->d_dx;
    A.order = b->d_order;
    A.t = b->d_t;
    A.tend = b->d_tend;
    A.queue = b->d_queue;
    A.cnt = b->d_cnt;
    A.T = b->T;
    A.nprob = b->nprob;
    A.ksteps = b->ksteps;
    A.cfl = cfl;
    A.e = b->eos;
    A.P = b->par;
    hipLaunchKernelGGL(hrm::k_set_int, dim3(1), dim3(64), 0, s, b->d_queue, 0);
    int rc = b->N == 2 ? launch_n<2>(b, A, s) : launch_n<3>(b, A, s);
    if (rc != HRM_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        snprintf(b->err, sizeof(b->err), "hrm_batch launch: %s", hipGetErrorString(e));
        return HRM_EDEVICE;
    }
    return HRM_OK;
}

void drop_graph(hrm_batch* b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
}

}  // namespace

extern "C" {

const char* hrm_batch_last_error(const hrm_batch* b) { return b ? b->err : "NULL batch"; }

int hrm_batch_create(const hrm_eos* e, const hrm_params* prm, int nprob, const long long* h_offsets,
                     const double* h_dx, int precision, hrm_batch** out)
{
    if (!out) return HRM_EINVAL;
    *out = nullptr;
    if (!e || !h_offsets || !h_dx || nprob < 1) return HRM_EINVAL;
    if (e->nspecies < 2 || e->nspecies > HRM_MAX_SPECIES) return HRM_EINVAL;
    for (int k = 0; k < e->nspecies; ++k) {
        if (!(e->gamma[k] > 1.0) || !(e->cv[k] > 0.0) || !(e->pinf[k] >= 0.0)) return HRM_EINVAL;
        if (k > 0 && e->pinf[k] != 0.0) return HRM_EINVAL;
    }
    if (precision != HRM_FP64 && precision != HRM_FP32) return HRM_EINVAL;
    if (e->nspecies != 2 && e->nspecies != 3) return HRM_EUNSUPPORTED;
    if (h_offsets[0] != 0) return HRM_EINVAL;
    for (int i = 0; i < nprob; ++i) {
        if (h_offsets[i + 1] <= h_offsets[i]) return HRM_EINVAL;  // every problem has >= 1 cell
        if (h_offsets[i + 1] - h_offsets[i] > (1ll << 30)) return HRM_EINVAL;
        if (!(h_dx[i] > 0.0)) return HRM_EINVAL;
    }
    hrm_batch* b = new (std::nothrow) hrm_batch;
    if (!b) return HRM_ENOMEM;
    memset(b, 0, sizeof(*b));
    b->N = e->nspecies;
    b->M = 2 * b->N + 1;
    b->nprob = nprob;
    b->precision = precision;
    b->T = h_offsets[nprob];
    for (int k = 0; k < hrm::MAXN; ++k) {
        const bool on = k < b->N;
        b->eos.g[k] = on ? e->gamma[k] : 2.0;
        b->eos.cv[k] = on ? e->cv[k] : 1.0;
        b->eos.pinf[k] = on ? e->pinf[k] : 0.0;
        b->eos.q[k] = on ? e->q[k] : 0.0;
        b->eos.ig1[k] = 1.0 / (b->eos.g[k] - 1.0);
        b->eos.gpi1[k] = b->eos.g[k] * b->eos.pinf[k] / (b->eos.g[k] - 1.0);
        b->eos.cp[k] = b->eos.g[k] * b->eos.cv[k];
    }
    hrm_params p;
    if (prm)
        p = *prm;
    else
        hrm_default_params(&p);
    hrm::ParDev& P = b->par;
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
    P.flags = 0;
    P.fast_flux_limiter = p.eps_f_ar >= p.hs_f_ar && p.eps_f_a >= p.hs_f_a && p.eps_f_re >= p.hs_f_re;
    // default launch: 256 threads, three workgroups per CU (the kernel's
    // register budget admits three waves per SIMD), 10 steps per launch
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    (void)hipGetLastError();
    b->threads = 256;
    b->blocks = 3 * cus;
    b->ksteps = 10;

    // longest problems first
    std::vector<int> order(nprob);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return h_offsets[x + 1] - h_offsets[x] > h_offsets[y + 1] - h_offsets[y];
    });
    const size_t bytes = sizeof(double) * (size_t)b->M * (size_t)b->T;
    bool ok = hipMalloc((void**)&b->d_W1, bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_W2, bytes) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_off, sizeof(long long) * (nprob + 1)) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_dx, sizeof(double) * nprob) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_order, sizeof(int) * nprob) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_t, sizeof(double) * nprob) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_tend, sizeof(double) * nprob) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_queue, sizeof(int)) == hipSuccess;
    ok = ok && hipMalloc((void**)&b->d_cnt, sizeof(unsigned long long) * 8) == hipSuccess;
    ok = ok && hipMemcpy(b->d_off, h_offsets, sizeof(long long) * (nprob + 1), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->d_dx, h_dx, sizeof(double) * nprob, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(b->d_order, order.data(), sizeof(int) * nprob, hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemset(b->d_t, 0, sizeof(double) * nprob) == hipSuccess;
    ok = ok && hipMemset(b->d_tend, 0, sizeof(double) * nprob) == hipSuccess;
    ok = ok && hipMemset(b->d_cnt, 0, sizeof(unsigned long long) * 8) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        hrm_batch_destroy(b);
        return HRM_ENOMEM;
    }
    *out = b;
    return HRM_OK;
}

int hrm_batch_destroy(hrm_batch* b)
{
    if (!b) return HRM_EINVAL;
    (void)hipDeviceSynchronize();
    drop_graph(b);
    (void)hipFree(b->d_W1);
    (void)hipFree(b->d_W2);
    (void)hipFree(b->d_off);
    (void)hipFree(b->d_dx);
    (void)hipFree(b->d_order);
    (void)hipFree(b->d_t);
    (void)hipFree(b->d_tend);
    (void)hipFree(b->d_queue);
    (void)hipFree(b->d_cnt);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    return HRM_OK;
}

int hrm_batch_configure(hrm_batch* b, int threads, int blocks, int steps_per_launch)
{
    if (!b) return HRM_EINVAL;
    if ((threads != 64 && threads != 128 && threads != 256) || blocks < 1 || blocks > 65536 || steps_per_launch < 1)
        return bfail(b, HRM_EINVAL, "hrm_batch_configure: threads in {64,128,256}, blocks >= 1, steps >= 1");
    if (threads != b->threads || blocks != b->blocks || steps_per_launch != b->ksteps) drop_graph(b);
    b->threads = threads;
    b->blocks = blocks;
    b->ksteps = steps_per_launch;
    return HRM_OK;
}

int hrm_batch_run(hrm_batch* b, double* d_W, int nsteps, double cfl, void* stream)
{
    if (!b) return HRM_EINVAL;
    if (!d_W || nsteps < 0 || !(cfl > 0.0)) return bfail(b, HRM_EINVAL, "hrm_batch_run: bad arguments");
    if (nsteps % b->ksteps != 0)
        return bfail(b, HRM_EINVAL, "hrm_batch_run: nsteps must be a multiple of the steps per launch");
    hipStream_t s = (hipStream_t)stream;
    b->last_stream = s;
    if (!b->gexec || b->g_W != d_W || b->g_cfl != cfl) {
        drop_graph(b);
        if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess)
            return bfail(b, HRM_EDEVICE, "hrm_batch_run: stream capture failed");
        const int rc = enqueue_chunk(b, d_W, cfl, b->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->cap_stream, &g);
        if (rc != HRM_OK || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return rc != HRM_OK ? rc : bfail(b, HRM_EDEVICE, "hrm_batch_run: end capture failed");
        }
        const hipError_t ei = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b->gexec = nullptr;
            return bfail(b, HRM_EDEVICE, "hrm_batch_run: graph instantiate failed");
        }
        b->g_W = d_W;
        b->g_cfl = cfl;
    }
    for (int k = 0; k < nsteps / b->ksteps; ++k)
        if (hipGraphLaunch(b->gexec, s) != hipSuccess) return bfail(b, HRM_EDEVICE, "hrm_batch_run: graph launch");
    return HRM_OK;
}

int hrm_batch_time(hrm_batch* b, double* h_t)
{
    if (!b || !h_t) return HRM_EINVAL;
    if (hipStreamSynchronize(b->last_stream) != hipSuccess ||
        hipMemcpy(h_t, b->d_t, sizeof(double) * b->nprob, hipMemcpyDeviceToHost) != hipSuccess)
        return bfail(b, HRM_EDEVICE, "hrm_batch_time: copy failed");
    return HRM_OK;
}

int hrm_batch_set_end_times(hrm_batch* b, const double* h_tend)
{
    if (!b || !h_tend) return HRM_EINVAL;
    for (int i = 0; i < b->nprob; ++i)
        if (!(h_tend[i] == h_tend[i])) return bfail(b, HRM_EINVAL, "hrm_batch_set_end_times: NaN end time");
    // ordered after the work already enqueued on the batch
    if (hipStreamSynchronize(b->last_stream) != hipSuccess ||
        hipMemcpy(b->d_tend, h_tend, sizeof(double) * b->nprob, hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, HRM_EDEVICE, "hrm_batch_set_end_times: copy failed");
    return HRM_OK;
}

int hrm_batch_get_diagnostics(hrm_batch* b, hrm_diag* out)
{
    if (!b || !out) return HRM_EINVAL;
    if (hipStreamSynchronize(b->last_stream) != hipSuccess ||
        hipMemcpy(out, b->d_cnt, sizeof(hrm_diag), hipMemcpyDeviceToHost) != hipSuccess)
        return bfail(b, HRM_EDEVICE, "hrm_batch_get_diagnostics: copy failed");
    return out->relax_bad ? HRM_EADMISSIBLE : HRM_OK;
}

}  // extern "C"
