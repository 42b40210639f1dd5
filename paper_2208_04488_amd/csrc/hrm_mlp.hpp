// hrm_mlp.hpp -- learned nonlinear interpolation weights on the matrix cores
// (gfx950 bfloat16 MFMA, float accumulation).
//
// An extension of the method (the paper's weights are those of App. C): the
// value at i+1/2 is a convex combination of the three 3-point candidates of
// the fifth-order interpolation from u_{i-2..i+2},
//   S_l = (3u_{i-2} - 10u_{i-1} + 15u_i)/8, S_c = (-u_{i-1} + 6u_i + 3u_{i+1})/8,
//   S_r = (3u_i + 6u_{i+1} - u_{i+2})/8,    linear weights d = (1/16, 10/16, 5/16),
// with omega_k proportional to d_k e^{tanh z_k} / (eps + beta_k)^2: the
// network's logits z rescale the classical WENO5 weights (Jiang & Shu
// smoothness indicators beta_k of the normalised stencil, eps = 1e-6) by at
// most e in either direction, so near a discontinuity the candidates that
// cross it keep negligible weights.  z comes from a 5-32-32-3 ReLU perceptron
// of the normalised stencil x_j = (u_j - u_i) r, r = 1 / max_j |u_j - u_i|.
// Parameters (1347 floats): W1[5][32], b1[32], W2[32][32], b2[32], W3[32][3],
// b3[3], rows indexed by the input unit.
//
// Evaluation: samples are matrix columns.  A wave evaluates 32 samples per
// 32x32x16 MFMA with the weights as the A operand (rows = output units) and
// the activations as the B operand (rows = input units).  The accumulator of
// one layer is the B operand of the next after a fixed renumbering of the
// hidden units, folded into the packed weights (see mlp_perm), so the hidden
// layers never leave the registers.  Inputs, W1, b1 (as the weight of a
// constant input 1), W2, W3 and both hidden activations are bfloat16 (round
// to nearest even); b2 initialises the layer-2 accumulator, b3 is added in
// float.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>

namespace hrm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ReLU of two floats, rounded to bfloat16 and packed.  Rounding to nearest
// keeps the sign, so the max with 0 can follow it, taken on the bfloat16
// bit patterns as 16-bit integers (the sign bit set means a negative
// integer, -0 and negative NaN included): one packed conversion and one
// packed integer max per pair, the same bits as the max before the rounding.
__device__ inline unsigned relu_bf16x2(float a, float b)
{
    const bf16x2 c = __builtin_convertvector((f32x2){a, b}, bf16x2);
    const i16x2 m = __builtin_elementwise_max(__builtin_bit_cast(i16x2, c), (i16x2)0);
    return __builtin_bit_cast(unsigned, m);
}

// ReLU of 8 accumulator entries, rounded to bfloat16
__device__ inline bf16x8 relu_bf16(const f32x16& acc, int base)
{
    u32x4 r;
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = relu_bf16x2(acc[base + 2 * q], acc[base + 2 * q + 1]);
    return __builtin_bit_cast(bf16x8, r);
}

constexpr int MLP_NPARAM = 1347;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = 160, MLP_OFF_W2 = 192, MLP_OFF_B2 = 1216, MLP_OFF_W3 = 1248,
              MLP_OFF_B3 = 1344;

// per-lane A-operand fragments (lane l holds row l % 32, K entries
// 8 (l / 32) .. 8 (l / 32) + 7 of each 16-deep K block)
struct MlpPacked {
    bf16x8 A1[64];     // layer 1: K = (x_0..x_4, 1, 0, 0) twice (K 0..7 and 8..15)
    bf16x8 A2[2][64];  // layer 2: two K blocks over the 32 hidden units
    bf16x8 A3[2][64];  // layer 3: rows 0..2 and again 4..6 are the logits, the rest zero
    float b2[32];
    float b3[4];
};

// Hidden unit fed as K index k of a layer: accumulator register v of lane
// (h = l / 32) holds row 8 (v / 4) + 4 h + v % 4; block kb of the next MFMA
// reads registers 8 kb .. 8 kb + 7 as K entries 16 kb + 8 h + q.
__host__ __device__ inline int mlp_perm(int k)
{
    const int kb = k >> 4, h = (k >> 3) & 1, q = k & 7;
    return 16 * kb + 8 * (q >> 2) + 4 * h + (q & 3);
}

// one 32-sample column block: xin = this lane's B entries of layer 1; the
// logits of column c are returned in lanes c and 32 + c (rows 0..2 and 4..6)
__device__ inline void mlp_block(const MlpPacked* __restrict__ m, const bf16x8 xin, float* z)
{
    const int lane = __lane_id();
    const int h = lane >> 5;
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m->A1[lane], xin, acc, 0, 0, 0);
    bf16x8 p0 = relu_bf16(acc, 0), p1 = relu_bf16(acc, 8);
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = m->b2[8 * (v >> 2) + 4 * h + (v & 3)];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m->A2[0][lane], p0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m->A2[1][lane], p1, acc, 0, 0, 0);
    p0 = relu_bf16(acc, 0);
    p1 = relu_bf16(acc, 8);
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m->A3[0][lane], p0, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(m->A3[1][lane], p1, acc, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 3; ++k) z[k] = acc[k] + m->b3[k];
}

// logits of this lane's sample x[5] (every lane of the wave takes part).
// Layer 1's weights fill both halves of K, so each lane feeds its own
// sample: lanes 0..31 as K 0..7 of the first block (lanes 32..63 zero),
// lanes 32..63 as K 8..15 of the second (lanes 0..31 zero).
__device__ inline void mlp_logits(const MlpPacked* __restrict__ m, const float* x, float* z)
{
    const bool lo = __lane_id() < 32;
    u32x4 xv;  // (x_0..x_4, 1, 0, 0) in bfloat16
    xv[0] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){x[0], x[1]}, bf16x2));
    xv[1] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){x[2], x[3]}, bf16x2));
    xv[2] = __builtin_bit_cast(unsigned, __builtin_convertvector((f32x2){x[4], 1.0f}, bf16x2));
    xv[3] = 0u;
    const u32x4 zero = {0u, 0u, 0u, 0u};
    const bf16x8 in0 = __builtin_bit_cast(bf16x8, lo ? xv : zero);
    const bf16x8 in1 = __builtin_bit_cast(bf16x8, lo ? zero : xv);
    float z0[3], z1[3];
    mlp_block(m, in0, z0);  // samples of lanes 0..31
    mlp_block(m, in1, z1);  // samples of lanes 32..63, in their own lanes
#pragma unroll
    for (int k = 0; k < 3; ++k) z[k] = lo ? z0[k] : z1[k];
}

constexpr float MLP_EPS = 1e-6f;  // of the classical weights, in normalised units

// smoothness indicators of the three candidates (Jiang & Shu) of x[0..4]
__host__ __device__ inline void mlp_beta(const float* x, float* b)
{
    const float a0 = x[0] - 2.0f * x[1] + x[2], c0 = x[0] - 4.0f * x[1] + 3.0f * x[2];
    const float a1 = x[1] - 2.0f * x[2] + x[3], c1 = x[1] - x[3];
    const float a2 = x[2] - 2.0f * x[3] + x[4], c2 = 3.0f * x[2] - 4.0f * x[3] + x[4];
    b[0] = 13.0f / 12.0f * a0 * a0 + 0.25f * c0 * c0;
    b[1] = 13.0f / 12.0f * a1 * a1 + 0.25f * c1 * c1;
    b[2] = 13.0f / 12.0f * a2 * a2 + 0.25f * c2 * c2;
}

// tanh(x) = 1 - 2/(e^{2x} + 1) from the hardware exponential and
// reciprocal: absolute error of a few 1e-8, which is what matters where the
// value is an exponent (large |x| gives +-1, NaN stays NaN)
__device__ inline float mlp_tanh(float x)
{
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * x) + 1.0f);
}

// omega_k = d_k e^{tanh z_k} / (eps + beta_k)^2, normalised: the network
// rescales each classical weight of the normalised stencil x by a factor in
// [1/e, e]; false if a weight is not finite.  Exponentials and reciprocals
// are the hardware ones (float, about an ulp): the weights are float anyway.
__device__ inline bool mlp_omega(const float* z, const float* x, float* w)
{
    float b[3];
    mlp_beta(x, b);
    const float t0 = mlp_tanh(z[0]), t1 = mlp_tanh(z[1]), t2 = mlp_tanh(z[2]);
    const float mx = fmaxf(t0, fmaxf(t1, t2));
    const float q0 = MLP_EPS + b[0], q1 = MLP_EPS + b[1], q2 = MLP_EPS + b[2];
    const float a0 = 0.0625f * __expf(t0 - mx) * __builtin_amdgcn_rcpf(q0 * q0);
    const float a1 = 0.625f * __expf(t1 - mx) * __builtin_amdgcn_rcpf(q1 * q1);
    const float a2 = 0.3125f * __expf(t2 - mx) * __builtin_amdgcn_rcpf(q2 * q2);
    const float is = __builtin_amdgcn_rcpf(a0 + a1 + a2);
    w[0] = a0 * is;
    w[1] = a1 * is;
    w[2] = a2 * is;
    return isfinite(w[0]) && isfinite(w[1]) && isfinite(w[2]);
}

// normalised float inputs of a stencil u[0..4] (u[2] the node i)
template <typename R>
__device__ inline void mlp_inputs(const R* u, float* x)
{
    R s = (R)0;
#pragma unroll
    for (int j = 0; j < 5; ++j) s = fmax(s, fabs(u[j] - u[2]));
    const R r = s > (R)0 ? (R)1 / s : (R)0;
#pragma unroll
    for (int j = 0; j < 5; ++j) x[j] = (float)((u[j] - u[2]) * r);
}

// sum_k w_k S_k written as S_c + w_l (S_l - S_c) + w_r (S_r - S_c): the
// weights sum to one only to float round-off, and this form keeps a constant
// stencil exact
template <typename R>
__device__ inline R mlp_value(const R* u, const float* w)
{
    const R sl = ((R)3 * u[0] - (R)10 * u[1] + (R)15 * u[2]) / (R)8;
    const R sc = (-u[1] + (R)6 * u[2] + (R)3 * u[3]) / (R)8;
    const R sr = ((R)3 * u[2] + (R)6 * u[3] - u[4]) / (R)8;
    return sc + (R)w[0] * (sl - sc) + (R)w[2] * (sr - sc);
}

// ---------------------------------------------------------------- host side
// float -> bfloat16 bits, round to nearest even (NaN kept quiet)
inline unsigned short host_bf16_bits(float f)
{
    unsigned int u;
    std::memcpy(&u, &f, sizeof(u));
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// parameters (1347 floats, layout above) -> per-lane MFMA fragments
inline void mlp_pack_host(const float* P, MlpPacked* out)
{
    std::memset(out, 0, sizeof(*out));
    auto put = [](bf16x8& dst, int q, float v) {
        unsigned short b = host_bf16_bits(v);
        std::memcpy(reinterpret_cast<unsigned char*>(&dst) + 2 * q, &b, 2);
    };
    for (int lane = 0; lane < 64; ++lane) {
        const int i = lane & 31, h = lane >> 5;
        for (int q = 0; q < 8; ++q) {
            // layer 1, both halves of K: inputs, then the constant input of b1
            const float a1 = q < 5 ? P[MLP_OFF_W1 + q * 32 + i] : (q == 5 ? P[MLP_OFF_B1 + i] : 0.0f);
            put(out->A1[lane], q, a1);
            for (int kb = 0; kb < 2; ++kb) {
                const int g = mlp_perm(16 * kb + 8 * h + q);
                put(out->A2[kb][lane], q, P[MLP_OFF_W2 + g * 32 + i]);
                const int o = i < 3 ? i : (i >= 4 && i < 7 ? i - 4 : -1);  // logit row
                put(out->A3[kb][lane], q, o >= 0 ? P[MLP_OFF_W3 + g * 3 + o] : 0.0f);
            }
        }
    }
    for (int i = 0; i < 32; ++i) out->b2[i] = P[MLP_OFF_B2 + i];
    for (int k = 0; k < 3; ++k) out->b3[k] = P[MLP_OFF_B3 + k];
}

}  // namespace hrm
