// Wave-wide evaluation of the surrogate networks on the matrix cores: per wave and
// stencil offset, 64 pair distances go through one network at once.  The 32 x 32
// middle layer of those 64 evaluations runs as Z2^T = W2 H1^T in two 32-column
// blocks (v_mfma_f32_32x32x8 bf16, float32 accumulation).  W2 is the A operand, held
// in registers; lanes l and l + 32 share a column and each computes the half of the
// first layer that its B-operand slots hold.  The bfloat16 B operands carry each
// activation as a sum of two bfloat16 terms.  Every lane of the wave must take part.
#pragma once

#include "misa_internal.h"

namespace misa {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_float(uint32_t b) { return __uint_as_float(b << 16); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));

// Two floats to packed bfloat16 (one v_cvt_pk_bf16_f32, round to nearest even).
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    const f32x2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// x = hi + lo with both terms bfloat16 (relative error of the pair ~2^-17).
__device__ __forceinline__ void split4(const float (&x)[4], bf16x4_t &hi, bf16x4_t &lo) {
    const uint32_t h01 = pk_bf16(x[0], x[1]), h23 = pk_bf16(x[2], x[3]);
    const uint32_t l01 = pk_bf16(x[0] - __uint_as_float(h01 << 16), x[1] - __uint_as_float(h01 & 0xffff0000u));
    const uint32_t l23 = pk_bf16(x[2] - __uint_as_float(h23 << 16), x[3] - __uint_as_float(h23 & 0xffff0000u));
    const uint2 hv = {h01, h23}, lv = {l01, l23};
    hi = __builtin_bit_cast(bf16x4_t, hv);
    lo = __builtin_bit_cast(bf16x4_t, lv);
}

// Per-unit constants of one network in LDS; float4 q covers units 4q .. 4q + 3.
struct MlpLds {
    float4 w1[8], b1[8], b2[8], w3[8];
    float b3;
};

__device__ __forceinline__ void fill_lds(MlpLds &L, const float *__restrict__ p) {
    const int i = threadIdx.x;
    if (i < MLP_H) {
        reinterpret_cast<float *>(L.w1)[i] = p[OFF_W1 + i];
        reinterpret_cast<float *>(L.b1)[i] = p[OFF_B1 + i];
        reinterpret_cast<float *>(L.b2)[i] = p[OFF_B2 + i];
        reinterpret_cast<float *>(L.w3)[i] = p[OFF_W3 + i];
    }
    if (i == 0) L.b3 = p[OFF_B3];
}

// A operand of K-step s for this lane: W2[unit = lane % 32][8 s + 4 h + i], i = 0..3.
__device__ __forceinline__ void load_a(bf16x4_t (&A)[4], const uint16_t *__restrict__ w2b) {
    const int lane = threadIdx.x & 63, h = lane >> 5, n = lane & 31;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const uint16_t *q = w2b + n * MLP_H + 8 * s + 4 * h;
#pragma unroll
        for (int i = 0; i < 4; ++i) A[s][i] = (short)q[i];
    }
}

// One 32-column block: column p = lane % 32 evaluates the network at t (lanes
// l and l ^ 32 pass the same t).  Returns the normalised y and dy/dt in both lanes.
// Accumulator element 4 j + i of lane l is row 8 j + 4 (l / 32) + i, column l % 32.
template <bool kTan>
__device__ __forceinline__ void mlp_block(const MlpLds &L, const bf16x4_t (&A)[4], float t, int h, float &y,
                                          float &dy) {
    f32x16_t acc, tac;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 b = L.b2[2 * j + h];
        acc[4 * j + 0] = b.x;
        acc[4 * j + 1] = b.y;
        acc[4 * j + 2] = b.z;
        acc[4 * j + 3] = b.w;
    }
    if (kTan)
#pragma unroll
        for (int v = 0; v < 16; ++v) tac[v] = 0.0f;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const float4 w = L.w1[2 * s + h], b = L.b1[2 * s + h];
        const float wv[4] = {w.x, w.y, w.z, w.w}, bv[4] = {b.x, b.y, b.z, b.w};
        float hv[4], dv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = wv[i] * t + bv[i];
            const float sg = sigm(z);
            hv[i] = z * sg;
            dv[i] = (sg + hv[i] * (1.0f - sg)) * wv[i];
        }
        bf16x4_t bh, bl;
        split4(hv, bh, bl);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A[s], bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A[s], bl, acc, 0, 0, 0);
        if (kTan) {
            bf16x4_t dh, dl;
            split4(dv, dh, dl);
            tac = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A[s], dh, tac, 0, 0, 0);
            tac = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(A[s], dl, tac, 0, 0, 0);
        }
    }
    float py = 0.0f, pd = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 w = L.w3[2 * j + h];
        const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = acc[4 * j + i];
            const float sg = sigm(z);
            const float hz = z * sg;
            py += wv[i] * hz;
            if (kTan) pd += wv[i] * (sg + hz * (1.0f - sg)) * tac[4 * j + i];
        }
    }
    py += __shfl_xor(py, 32);
    y = py + L.b3;
    if (kTan) {
        pd += __shfl_xor(pd, 32);
        dy = pd;
    }
}

// The network at one normalised input per lane (all 64 lanes must take part).
template <bool kTan>
__device__ __forceinline__ void mlp_wave(const MlpLds &L, const bf16x4_t (&A)[4], float t_own, float &y,
                                         float &dy) {
    const int h = (threadIdx.x >> 5) & 1;
    const float t_par = __shfl_xor(t_own, 32);
    float y0, d0 = 0.0f, y1, d1 = 0.0f;
    mlp_block<kTan>(L, A, h ? t_par : t_own, h, y0, d0);  // columns = pairs of lanes 0..31
    mlp_block<kTan>(L, A, h ? t_own : t_par, h, y1, d1);  // columns = pairs of lanes 32..63
    y = h ? y1 : y0;
    dy = h ? d1 : d0;
}

__device__ __forceinline__ float net_t(const MlpNet &m, float x) {
    return (fminf(fmaxf(x, m.x_lo), m.x_hi) - m.c) * m.s;
}

// float32 table fall-back outside a network's range (the records of the float32 form)
__device__ __forceinline__ void seg32(float x, const TabMeta<float> &m, int &k, float &t) {
    const float p = (x - m.x0) * m.inv_h;
    int kk = (int)p;
    kk = kk < m.nseg - 1 ? kk : m.nseg - 1;
    kk = kk > 0 ? kk : 0;
    k = kk;
    t = p - (float)kk;
}

__device__ __forceinline__ float emb_tab(float rho, const Tables<float> &T, float &Fv, bool &beyond) {
    const TabMeta<float> &m = T.em;
    if (rho > m.x_last) {
        beyond = true;
        Fv = m.y_last + m.d_last * (rho - m.x_last);
        return m.d_last;
    }
    int k;
    float t;
    seg32(rho, m, k, t);
    const Q4<float> c = T.emb[2 * k], d = T.emb[2 * k + 1];
    Fv = ((c.w * t + c.z) * t + c.y) * t + c.x;
    return (d.z * t + d.y) * t + d.x;
}

}  // namespace misa
