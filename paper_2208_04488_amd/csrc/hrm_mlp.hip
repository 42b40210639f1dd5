// hrm_mlp.hip -- training of the learned interpolation weights on the GPU
// (gfx950): extraction of training pairs from a fine ensemble, float32
// forward + backward pass with per-workgroup gradient sums, a fixed-order
// reduction and the Adam update.  Declarations and semantics: include/hrm.h.
//
// The network and the interpolant are described in hrm_mlp.hpp.  Training
// runs in float32 on the vector ALUs (the matrix-core evaluation in bfloat16
// is for inference inside the solver): a minibatch has at most a few hundred
// thousand samples and 1347 parameters, far from any roofline that matters.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "hrm.h"
#include "hrm_face.hpp"

namespace hrm {

constexpr int TR_BLOCK = 64;               // samples per workgroup (one wave)
constexpr int TR_PARTIAL = MLP_NPARAM + 1;  // gradient entries + loss

// ---------------------------------------------------------------- extraction
template <int N>
struct ExtractArgs {
    const double* W;
    long long T;
    const long long* off;   // fine offsets (nprob + 1)
    const long long* soff;  // first sample of each problem (nprob + 1)
    float* X;               // nsamp x 8 (x_0..x_4, 0, 0, 0)
    float* Tt;              // nsamp
    EosDev e;
};

// field f of the 1D primitive vector (alpha_k rho_k, u, p, alpha_k) at fine cell g
template <int N>
__device__ inline double prim_field(const ExtractArgs<N>& A, long long g, int f)
{
    constexpr int M = 2 * N + 1;
    double w[M];
#pragma unroll
    for (int c = 0; c < M; ++c) w[c] = A.W[c * A.T + g];
    if (f < N) return w[f];
    if (f >= N + 2) return w[f];  // alpha_k sits in the same slot of W and V
    St<N, 1> s;
    state_from_W<N, 1>(A.e, w, s);
    return f == N ? s.u[0] : s.p;
}

// one workgroup per problem: coarse node j = fine node 2j; for field f the
// left-biased pairs (coarse j-2..j+2, label fine 2j+1) for j = 2..n-3, then
// the mirrored ones (coarse j+3..j-1, same label) for j = 1..n-4
template <int N>
__global__ void __launch_bounds__(256) k_mlp_extract(const ExtractArgs<N> A)
{
    constexpr int M = 2 * N + 1;
    const int b = blockIdx.x;
    const long long base = A.off[b];
    const long long nf = A.off[b + 1] - base;
    const long long n = nf / 2;
    if (nf % 2 != 0 || n < 5) return;
    const long long per = n - 4, total = (long long)M * 2 * per;
    for (long long q = threadIdx.x; q < total; q += blockDim.x) {
        const int f = (int)(q / (2 * per));
        const long long r = q % (2 * per);
        const bool right = r >= per;
        const long long j = right ? 1 + (r - per) : 2 + r;
        double u[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const long long cj = right ? j + 3 - i : j - 2 + i;
            u[i] = prim_field<N>(A, base + 2 * cj, f);
        }
        const double label = prim_field<N>(A, base + 2 * j + 1, f);
        double s = 0.0, amax = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            s = fmax(s, fabs(u[i] - u[2]));
            amax = fmax(amax, fabs(u[i]));
        }
        // variations at round-off level carry no shape, and a label outside
        // [-4, 4] in normalised units (a feature the coarse stencil does not
        // see) lies beyond every convex combination of the candidates
        // (|S_k| <= 3.5): such pairs are neutral
        double rr = s > 1e-10 * amax ? 1.0 / s : 0.0;
        if (!(fabs((label - u[2]) * rr) <= 4.0)) rr = 0.0;
        const long long out = A.soff[b] + q;
#pragma unroll
        for (int i = 0; i < 5; ++i) A.X[out * 8 + i] = (float)((u[i] - u[2]) * rr);
        A.X[out * 8 + 5] = 0.0f;
        A.X[out * 8 + 6] = 0.0f;
        A.X[out * 8 + 7] = 0.0f;
        A.Tt[out] = (float)((label - u[2]) * rr);
    }
}

// Pairs from a fine grid: lines along each direction d (those with an even
// number of fine cells 2n, n >= 5), one line per `st`-th fine cell in each
// transverse direction, with the recipe of k_mlp_extract on every line and
// every field of the primitive vector (alpha_k rho_k, u_d, p, alpha_k).
template <int N, int D>
struct GridExtractArgs {
    const double* W;
    long long nc;
    int n[3];
    int st;
    long long first_line[4];  // index of the first line of each direction (first_line[3] = all lines)
    long long base[3];        // first sample of each direction
    long long per[3];         // samples per line of each direction
    int nta[3];               // sampled transverse positions along the first transverse dimension
    float* X;
    float* Tt;
    EosDev e;
};

// field f of the primitive vector (alpha_k rho_k, u_d, p, alpha_k) of a cell
template <int N, int D>
__device__ inline double grid_prim(const GridExtractArgs<N, D>& A, long long cell, int f)
{
    constexpr int M = 2 * N + D;
    double w[M];
#pragma unroll
    for (int c = 0; c < M; ++c) w[c] = A.W[c * A.nc + cell];
    if (f < N || f > N + D) return w[f];  // partial densities; alpha_k sit in the same slots of W and V
    St<N, D> s;
    state_from_W<N, D>(A.e, w, s);
    return f < N + D ? s.u[f - N] : s.p;
}

// one workgroup per line
template <int N, int D>
__global__ void __launch_bounds__(256) k_mlp_extract_grid(const GridExtractArgs<N, D> A)
{
    constexpr int M = 2 * N + D;
    const long long L = blockIdx.x;
    const int d = L < A.first_line[1] ? 0 : (L < A.first_line[2] ? 1 : 2);
    const long long li = L - A.first_line[d];
    const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;  // transverse dimensions
    const long long ia = (li % A.nta[d]) * A.st, ib = (li / A.nta[d]) * A.st;
    const long long stride[3] = {1, A.n[0], (long long)A.n[0] * A.n[1]};
    const long long line0 = ia * stride[ta] + ib * stride[tb];
    const long long sd = stride[d];
    const long long n = A.n[d] / 2;
    const long long per = n - 4;
    for (long long q = threadIdx.x; q < A.per[d]; q += blockDim.x) {
        const int f = (int)(q / (2 * per));
        const long long r = q % (2 * per);
        const bool right = r >= per;
        const long long j = right ? 1 + (r - per) : 2 + r;
        double u[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const long long cj = right ? j + 3 - i : j - 2 + i;
            u[i] = grid_prim<N, D>(A, line0 + 2 * cj * sd, f);
        }
        const double label = grid_prim<N, D>(A, line0 + (2 * j + 1) * sd, f);
        double s = 0.0, amax = 0.0;
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            s = fmax(s, fabs(u[i] - u[2]));
            amax = fmax(amax, fabs(u[i]));
        }
        double rr = s > 1e-10 * amax ? 1.0 / s : 0.0;
        if (!(fabs((label - u[2]) * rr) <= 4.0)) rr = 0.0;
        const long long out = A.base[d] + li * A.per[d] + q;
#pragma unroll
        for (int i = 0; i < 5; ++i) A.X[out * 8 + i] = (float)((u[i] - u[2]) * rr);
        A.X[out * 8 + 5] = 0.0f;
        A.X[out * 8 + 6] = 0.0f;
        A.X[out * 8 + 7] = 0.0f;
        A.Tt[out] = (float)((label - u[2]) * rr);
    }
    (void)M;
}

// ---------------------------------------------------------------- gradient
struct GradArgs {
    const float* P;
    const float* X;
    const float* Tt;
    long long nsamp, first, stride;
    int count;
    float* partial;  // gridDim.x x TR_PARTIAL
};

__global__ void __launch_bounds__(TR_BLOCK) k_mlp_grad(const GradArgs A)
{
    __shared__ float sP[MLP_NPARAM];
    __shared__ float sx[TR_BLOCK][5], sh1[TR_BLOCK][33], sdh1[TR_BLOCK][33], sh2[TR_BLOCK][33],
        sdh2[TR_BLOCK][33], sdz[TR_BLOCK][3], sl[TR_BLOCK];
    const int t = threadIdx.x;
    for (int i = t; i < MLP_NPARAM; i += TR_BLOCK) sP[i] = A.P[i];
    __syncthreads();
    const float* W1 = sP + MLP_OFF_W1;
    const float* b1 = sP + MLP_OFF_B1;
    const float* W2 = sP + MLP_OFF_W2;
    const float* b2 = sP + MLP_OFF_B2;
    const float* W3 = sP + MLP_OFF_W3;
    const float* b3 = sP + MLP_OFF_B3;

    const long long k = (long long)blockIdx.x * TR_BLOCK + t;
    const bool on = k < A.count;
    float x[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, tt = 0.0f;
    if (on) {
        const long long idx = (A.first + k * A.stride) % A.nsamp;
#pragma unroll
        for (int j = 0; j < 5; ++j) x[j] = A.X[idx * 8 + j];
        tt = A.Tt[idx];
    }
    // forward
    float h1[32], h2[32];
#pragma unroll
    for (int h = 0; h < 32; ++h) {
        float a = b1[h];
#pragma unroll
        for (int j = 0; j < 5; ++j) a += x[j] * W1[j * 32 + h];
        h1[h] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int h = 0; h < 32; ++h) {
        float a = b2[h];
#pragma unroll
        for (int g = 0; g < 32; ++g) a += h1[g] * W2[g * 32 + h];
        h2[h] = fmaxf(a, 0.0f);
    }
    float z[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float a = b3[c];
#pragma unroll
        for (int h = 0; h < 32; ++h) a += h2[h] * W3[h * 3 + c];
        z[c] = a;
    }
    // weights: the classical ones of x rescaled by e^{tanh z_k}
    float bt[3], th[3];
    mlp_beta(x, bt);
#pragma unroll
    for (int c = 0; c < 3; ++c) th[c] = tanhf(z[c]);
    const float my = fmaxf(th[0], fmaxf(th[1], th[2]));
    const float dk[3] = {0.0625f, 0.625f, 0.3125f};
    float a[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float q = MLP_EPS + bt[c];
        a[c] = dk[c] * expf(th[c] - my) / (q * q);
    }
    const float ie = 1.0f / (a[0] + a[1] + a[2]);
    const float w[3] = {a[0] * ie, a[1] * ie, a[2] * ie};
    const float S[3] = {(3.0f * x[0] - 10.0f * x[1] + 15.0f * x[2]) * 0.125f,
                        (-x[1] + 6.0f * x[2] + 3.0f * x[3]) * 0.125f,
                        (3.0f * x[2] + 6.0f * x[3] - x[4]) * 0.125f};
    const float res = w[0] * S[0] + w[1] * S[1] + w[2] * S[2] - tt;
    // backward of the mean squared residual over the minibatch
    const float dy = on ? 2.0f * res / (float)A.count : 0.0f;
    const float dw[3] = {dy * S[0], dy * S[1], dy * S[2]};
    const float wdw = w[0] * dw[0] + w[1] * dw[1] + w[2] * dw[2];
    float dz[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) dz[c] = w[c] * (dw[c] - wdw) * (1.0f - th[c] * th[c]);
    float dh2[32], dh1[32];
#pragma unroll
    for (int h = 0; h < 32; ++h) {
        const float a = W3[h * 3 + 0] * dz[0] + W3[h * 3 + 1] * dz[1] + W3[h * 3 + 2] * dz[2];
        dh2[h] = h2[h] > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int g = 0; g < 32; ++g) {
        float a = 0.0f;
#pragma unroll
        for (int h = 0; h < 32; ++h) a += W2[g * 32 + h] * dh2[h];
        dh1[g] = h1[g] > 0.0f ? a : 0.0f;
    }
    // stage the activations and sum the outer products over the samples
#pragma unroll
    for (int j = 0; j < 5; ++j) sx[t][j] = x[j];
#pragma unroll
    for (int h = 0; h < 32; ++h) {
        sh1[t][h] = h1[h];
        sdh1[t][h] = dh1[h];
        sh2[t][h] = h2[h];
        sdh2[t][h] = dh2[h];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) sdz[t][c] = dz[c];
    sl[t] = on ? res * res : 0.0f;
    __syncthreads();
    float* out = A.partial + (size_t)blockIdx.x * TR_PARTIAL;
    for (int p = t; p < TR_PARTIAL; p += TR_BLOCK) {
        float acc = 0.0f;
        if (p < MLP_OFF_B1) {
            const int j = p / 32, h = p % 32;
            for (int s = 0; s < TR_BLOCK; ++s) acc += sx[s][j] * sdh1[s][h];
        } else if (p < MLP_OFF_W2) {
            const int h = p - MLP_OFF_B1;
            for (int s = 0; s < TR_BLOCK; ++s) acc += sdh1[s][h];
        } else if (p < MLP_OFF_B2) {
            const int g = (p - MLP_OFF_W2) / 32, h = (p - MLP_OFF_W2) % 32;
            for (int s = 0; s < TR_BLOCK; ++s) acc += sh1[s][g] * sdh2[s][h];
        } else if (p < MLP_OFF_W3) {
            const int h = p - MLP_OFF_B2;
            for (int s = 0; s < TR_BLOCK; ++s) acc += sdh2[s][h];
        } else if (p < MLP_OFF_B3) {
            const int h = (p - MLP_OFF_W3) / 3, c = (p - MLP_OFF_W3) % 3;
            for (int s = 0; s < TR_BLOCK; ++s) acc += sh2[s][h] * sdz[s][c];
        } else if (p < MLP_NPARAM) {
            const int c = p - MLP_OFF_B3;
            for (int s = 0; s < TR_BLOCK; ++s) acc += sdz[s][c];
        } else {
            for (int s = 0; s < TR_BLOCK; ++s) acc += sl[s];
        }
        out[p] = acc;
    }
}

// fixed-order sum of the workgroup partials (double accumulation): a
// workgroup takes RD_P entries, RD_S threads per entry each sum every RD_S-th
// partial in order, then the RD_S sums are added in order
constexpr int RD_P = 16, RD_S = 16;
__global__ void __launch_bounds__(RD_P* RD_S) k_mlp_reduce(const float* partial, int nblk, int count, float* grad,
                                                          float* loss)
{
    __shared__ double sh[RD_S][RD_P];
    const int pl = threadIdx.x % RD_P, part = threadIdx.x / RD_P;
    const int p = blockIdx.x * RD_P + pl;
    double acc = 0.0;
    if (p < TR_PARTIAL) {
#pragma unroll 8
        for (int b = part; b < nblk; b += RD_S) acc += (double)partial[(size_t)b * TR_PARTIAL + p];
    }
    sh[part][pl] = acc;
    __syncthreads();
    if (part == 0 && p < TR_PARTIAL) {
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < RD_S; ++k) sum += sh[k][pl];
        if (p < MLP_NPARAM)
            grad[p] = (float)sum;
        else
            *loss = (float)(sum / count);
    }
}

__global__ void __launch_bounds__(256) k_mlp_adam(float* P, const float* g, float* m, float* v, float lr, float b1,
                                                  float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    P[p] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline void fill_eos(const hrm_eos* e, int N, EosDev& o)
{
    for (int k = 0; k < MAXN; ++k) {
        const bool on = k < N;
        o.g[k] = on ? e->gamma[k] : 2.0;
        o.cv[k] = on ? e->cv[k] : 1.0;
        o.pinf[k] = on ? e->pinf[k] : 0.0;
        o.q[k] = on ? e->q[k] : 0.0;
        o.ig1[k] = 1.0 / (o.g[k] - 1.0);
        o.gpi1[k] = o.g[k] * o.pinf[k] / (o.g[k] - 1.0);
        o.cp[k] = o.g[k] * o.cv[k];
    }
}

// line and sample layout of the grid extraction (no device work)
struct GridLayout {
    long long first_line[4], base[3], per[3], total;
    int nta[3];
};

inline GridLayout grid_layout(const hrm_grid* g, int N, int st)
{
    GridLayout o;
    memset(&o, 0, sizeof(o));
    const int M = 2 * N + g->dim;
    long long line = 0, samp = 0;
    for (int d = 0; d < 3; ++d) {
        o.first_line[d] = line;
        o.base[d] = samp;
        const int ta = d == 0 ? 1 : 0, tb = d == 2 ? 1 : 2;
        const long long nf = g->n[d], nh = nf / 2;
        if (d < g->dim && nf % 2 == 0 && nh >= 5) {
            o.nta[d] = (g->n[ta] + st - 1) / st;
            const long long lines = (long long)o.nta[d] * ((g->n[tb] + st - 1) / st);
            o.per[d] = (long long)M * 2 * (nh - 4);
            line += lines;
            samp += lines * o.per[d];
        } else {
            o.nta[d] = 1;
        }
    }
    o.first_line[3] = line;
    o.total = samp;
    return o;
}

template <int N, int D>
int extract_grid_launch(const hrm_grid* g, const hrm_eos* e, const GridLayout& lay, int st, const double* d_W,
                        float* d_X, float* d_T, hipStream_t s)
{
    GridExtractArgs<N, D> A;
    memset(&A, 0, sizeof(A));
    A.W = d_W;
    A.nc = (long long)g->n[0] * g->n[1] * g->n[2];
    for (int d = 0; d < 3; ++d) {
        A.n[d] = g->n[d];
        A.base[d] = lay.base[d];
        A.per[d] = lay.per[d];
        A.nta[d] = lay.nta[d];
    }
    for (int d = 0; d < 4; ++d) A.first_line[d] = lay.first_line[d];
    A.st = st;
    A.X = d_X;
    A.Tt = d_T;
    fill_eos(e, N, A.e);
    hipLaunchKernelGGL((k_mlp_extract_grid<N, D>), dim3((unsigned)lay.first_line[3]), dim3(256), 0, s, A);
    return hipGetLastError() == hipSuccess ? HRM_OK : HRM_EDEVICE;
}

template <int N>
int extract_launch(const hrm_eos* e, const double* d_W, long long T, int nprob, const long long* d_off,
                   const long long* d_soff, float* d_X, float* d_T, hipStream_t s)
{
    ExtractArgs<N> A;
    memset(&A, 0, sizeof(A));
    A.W = d_W;
    A.T = T;
    A.off = d_off;
    A.soff = d_soff;
    A.X = d_X;
    A.Tt = d_T;
    fill_eos(e, N, A.e);
    hipLaunchKernelGGL(k_mlp_extract<N>, dim3(nprob), dim3(256), 0, s, A);
    return hipGetLastError() == hipSuccess ? HRM_OK : HRM_EDEVICE;
}

// largest minibatch of hrm_mlp_grad_noalloc and the floats of its partials
constexpr long long NOALLOC_FLOATS =
    (long long)((HRM_MLP_GRAD_NOALLOC_MAX + TR_BLOCK - 1) / TR_BLOCK) * TR_PARTIAL;

}  // namespace hrm

// The per-workgroup partial sums of hrm_mlp_grad_noalloc: a fixed array in
// device memory (one copy per device, held until the process ends).  In host
// code this name is not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
static __device__ __align__(256) float scratch[hrm::NOALLOC_FLOATS];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float* g_scratch[MAX_DEVICES] = {};

// address of `scratch` on the current device, looked up once per device
int noalloc_scratch(float** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return HRM_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return HRM_EDEVICE;
        }
        g_scratch[dev] = static_cast<float*>(p);
    }
    *out = g_scratch[dev];
    return HRM_OK;
}

// the two launches of a gradient: partials of every workgroup into `work`
// (each entry written before it is read), then their fixed-order sum
int grad_launch(const float* d_params, const float* d_X, const float* d_T, long long nsamp, long long first,
                long long stride, int count, float* d_grad, float* d_loss, float* work, hipStream_t s)
{
    hrm::GradArgs A;
    A.P = d_params;
    A.X = d_X;
    A.Tt = d_T;
    A.nsamp = nsamp;
    A.first = first % nsamp;
    A.stride = stride % nsamp == 0 ? 1 : stride % nsamp;
    A.count = count;
    A.partial = work;
    const int nblk = (count + hrm::TR_BLOCK - 1) / hrm::TR_BLOCK;
    hipLaunchKernelGGL(hrm::k_mlp_grad, dim3(nblk), dim3(hrm::TR_BLOCK), 0, s, A);
    hipLaunchKernelGGL(hrm::k_mlp_reduce, dim3((hrm::TR_PARTIAL + hrm::RD_P - 1) / hrm::RD_P),
                       dim3(hrm::RD_P * hrm::RD_S), 0, s, work, nblk, count, d_grad, d_loss);
    return hipGetLastError() == hipSuccess ? HRM_OK : HRM_EDEVICE;
}

}  // namespace

extern "C" {

int hrm_mlp_extract(const hrm_eos* e, const double* d_W, long long T, int nprob, const long long* h_offsets,
                    float* d_X, float* d_T, long long capacity, long long* nsamples, void* stream)
{
    if (!e || !h_offsets || !nsamples || nprob < 1 || T < 0) return HRM_EINVAL;
    if (e->nspecies != 2 && e->nspecies != 3) return HRM_EUNSUPPORTED;
    for (int k = 0; k < e->nspecies; ++k)
        if (!(e->gamma[k] > 1.0) || !(e->cv[k] > 0.0) || !(e->pinf[k] >= 0.0)) return HRM_EINVAL;
    if (h_offsets[0] != 0 || h_offsets[nprob] != T) return HRM_EINVAL;
    const int M = 2 * e->nspecies + 1;
    std::vector<long long> soff(nprob + 1, 0);
    for (int b = 0; b < nprob; ++b) {
        const long long nf = h_offsets[b + 1] - h_offsets[b];
        if (nf < 1) return HRM_EINVAL;
        const long long n = nf / 2;
        const long long cnt = (nf % 2 == 0 && n >= 5) ? (long long)M * 2 * (n - 4) : 0;
        soff[b + 1] = soff[b] + cnt;
    }
    *nsamples = soff[nprob];
    if (!d_X && !d_T) return HRM_OK;  // size query
    if (!d_W || !d_X || !d_T || capacity < soff[nprob]) return HRM_EINVAL;
    long long *d_off = nullptr, *d_soff = nullptr;
    hipStream_t s = (hipStream_t)stream;
    bool ok = hipMalloc((void**)&d_off, sizeof(long long) * (nprob + 1)) == hipSuccess;
    ok = ok && hipMalloc((void**)&d_soff, sizeof(long long) * (nprob + 1)) == hipSuccess;
    ok = ok && hipMemcpy(d_off, h_offsets, sizeof(long long) * (nprob + 1), hipMemcpyHostToDevice) == hipSuccess;
    ok = ok && hipMemcpy(d_soff, soff.data(), sizeof(long long) * (nprob + 1), hipMemcpyHostToDevice) == hipSuccess;
    int rc = ok ? HRM_OK : HRM_ENOMEM;
    if (rc == HRM_OK)
        rc = e->nspecies == 2 ? hrm::extract_launch<2>(e, d_W, T, nprob, d_off, d_soff, d_X, d_T, s)
                              : hrm::extract_launch<3>(e, d_W, T, nprob, d_off, d_soff, d_X, d_T, s);
    if (hipStreamSynchronize(s) != hipSuccess && rc == HRM_OK) rc = HRM_EDEVICE;
    (void)hipFree(d_off);
    (void)hipFree(d_soff);
    return rc;
}

int hrm_mlp_extract_grid(const hrm_grid* g, const hrm_eos* e, const double* d_W, int stride, float* d_X, float* d_T,
                         long long capacity, long long* nsamples, void* stream)
{
    if (!g || !e || !nsamples || stride < 1) return HRM_EINVAL;
    if (g->dim < 1 || g->dim > 3) return HRM_EINVAL;
    for (int d = 0; d < 3; ++d)
        if (g->n[d] < 1 || (d >= g->dim && g->n[d] != 1)) return HRM_EINVAL;
    if (e->nspecies != 2 && e->nspecies != 3) return HRM_EUNSUPPORTED;
    for (int k = 0; k < e->nspecies; ++k)
        if (!(e->gamma[k] > 1.0) || !(e->cv[k] > 0.0) || !(e->pinf[k] >= 0.0)) return HRM_EINVAL;
    const hrm::GridLayout lay = hrm::grid_layout(g, e->nspecies, stride);
    *nsamples = lay.total;
    if (!d_X && !d_T) return HRM_OK;  // size query
    if (!d_W || !d_X || !d_T || capacity < lay.total) return HRM_EINVAL;
    if (lay.first_line[3] > 0x7fffffffLL) return HRM_EUNSUPPORTED;
    if (lay.total == 0) return HRM_OK;
    hipStream_t s = (hipStream_t)stream;
    int rc = HRM_EUNSUPPORTED;
    switch (e->nspecies * 10 + g->dim) {
    case 21: rc = hrm::extract_grid_launch<2, 1>(g, e, lay, stride, d_W, d_X, d_T, s); break;
    case 22: rc = hrm::extract_grid_launch<2, 2>(g, e, lay, stride, d_W, d_X, d_T, s); break;
    case 23: rc = hrm::extract_grid_launch<2, 3>(g, e, lay, stride, d_W, d_X, d_T, s); break;
    case 31: rc = hrm::extract_grid_launch<3, 1>(g, e, lay, stride, d_W, d_X, d_T, s); break;
    case 32: rc = hrm::extract_grid_launch<3, 2>(g, e, lay, stride, d_W, d_X, d_T, s); break;
    case 33: rc = hrm::extract_grid_launch<3, 3>(g, e, lay, stride, d_W, d_X, d_T, s); break;
    default: break;
    }
    return rc;
}

long long hrm_mlp_grad_workspace(int count)
{
    return count < 1 ? 0 : (long long)((count + hrm::TR_BLOCK - 1) / hrm::TR_BLOCK) * hrm::TR_PARTIAL;
}

int hrm_mlp_grad(const float* d_params, const float* d_X, const float* d_T, long long nsamp, long long first,
                 long long stride, int count, float* d_grad, float* d_loss, float* d_work, long long work_floats,
                 void* stream)
{
    if (!d_params || !d_X || !d_T || !d_grad || !d_loss || !d_work) return HRM_EINVAL;
    if (nsamp < 1 || count < 1 || first < 0 || stride < 1) return HRM_EINVAL;
    if (work_floats < hrm_mlp_grad_workspace(count)) return HRM_EINVAL;
    return grad_launch(d_params, d_X, d_T, nsamp, first, stride, count, d_grad, d_loss, d_work, (hipStream_t)stream);
}

int hrm_mlp_grad_noalloc(const float* d_params, const float* d_X, const float* d_T, long long nsamp,
                         long long first, long long stride, int count, float* d_grad, float* d_loss, void* stream)
{
    if (!d_params || !d_X || !d_T || !d_grad || !d_loss) return HRM_EINVAL;
    if (nsamp < 1 || count < 1 || first < 0 || stride < 1) return HRM_EINVAL;
    if (count > HRM_MLP_GRAD_NOALLOC_MAX) return HRM_EINVAL;
    float* work = nullptr;
    if (const int rc = noalloc_scratch(&work)) return rc;
    return grad_launch(d_params, d_X, d_T, nsamp, first, stride, count, d_grad, d_loss, work, (hipStream_t)stream);
}

int hrm_mlp_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, int step, float lr, float beta1,
                 float beta2, float eps, void* stream)
{
    if (!d_params || !d_grad || !d_m || !d_v || step < 1) return HRM_EINVAL;
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return HRM_EINVAL;
    // bias corrections 1 - beta^step, formed in double
    double p1 = 1.0, p2 = 1.0;
    for (int i = 0; i < step && i < 100000; ++i) {
        p1 *= beta1;
        p2 *= beta2;
    }
    const float c1 = (float)(1.0 - p1), c2 = (float)(1.0 - p2);
    hipLaunchKernelGGL(hrm::k_mlp_adam, dim3((hrm::MLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       d_params, d_grad, d_m, d_v, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? HRM_OK : HRM_EDEVICE;
}

}  // extern "C"
