// Learned non-reflecting boundary closure: a small MLP evaluated and trained on matrix cores.
//
// Not in the paper (its domains are periodic).  The network maps the strip of post-collision
// populations at a face node (3 cells deep along the inward normal, Q values each, in the
// canonical face frame) to the k populations that enter the box through the face:
//   s = rms(x), z = x / s, h1 = relu(z W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3,
//   prediction = s y;  s is computed as m sqrt(mean((x/m)^2)), m = max |x|, so tiny strips do
//   not underflow; an all-zero strip has s = 0, z = 0 and predicts 0.
// Parameters are FP32 (master copy, layout W1[n_in][64], b1[64], W2[64][64], b2[64],
// W3[64][k], b3[k], row-major).  Every matrix product takes bfloat16 inputs (round to
// nearest even) and accumulates in FP32 on the matrix cores; biases are added in FP32.  The
// forward pass reduces over 32 values per instruction (v_mfma_f32_16x16x32_bf16, gfx950), the
// input padded with zeros to a multiple of 32 (a 16-wide product accumulated onto a 32-wide one's
// result gave wrong rows in this compiler's code, measured on D3Q7 and D3Q13, so every product of
// the forward pass has the one shape); the backward pass reduces over the 16 samples of a tile or
// over the hidden width with v_mfma_f32_16x16x16_bf16.
//
// One wave owns a tile of 16 samples.  MFMA operand layouts (lane l, element e; measured for
// 16x16x32 with an exact integer product on one wave):
//   16x16x16: A (16 x 16, rows i, reduction k): A[l % 16][4 (l / 16) + e]     (e < 4)
//             B (16 x 16, reduction k, cols j): B[4 (l / 16) + e][l % 16]
//   16x16x32: A (16 x 32): A[l % 16][8 (l / 16) + e], B (32 x 16): B[8 (l / 16) + e][l % 16]  (e < 8)
//   both:     C (16 x 16): C[4 (l / 16) + e][l % 16]
// Activations pass between layers through LDS (a per-wave [16][64] bfloat16 tile).
#pragma once

#include <hip/hip_runtime.h>

#include "velsets.hpp"

namespace lbm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kHidden = 64;

__device__ __forceinline__ unsigned short bf16_bits(float v) {
    unsigned u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

__device__ __forceinline__ floatx4 mfma16(bf16x4 a, bf16x4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma32(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a), __builtin_bit_cast(bf16x8v, b), c,
                                                   0, 0, 0);
}

// Wave-local LDS ordering: the wave's LDS accesses complete in program order; the fences
// keep the compiler from moving loads above the stores other lanes depend on.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of canonical entering populations (c_x = +1) of a velocity set.
template <class VS>
__host__ __device__ constexpr int entering_count() {
    int k = 0;
    for (int i = 0; i < VS::Q; ++i) k += VS::c[i][0] == 1 ? 1 : 0;
    return k;
}
template <class VS>
__host__ __device__ constexpr int entering_index(int r) {
    int k = 0;
    for (int i = 0; i < VS::Q; ++i)
        if (VS::c[i][0] == 1) {
            if (k == r) return i;
            ++k;
        }
    return -1;
}

// Time levels of the strip in the network input: the current step's and the previous step's.
constexpr int kHistory = 2;

template <class VS>
struct NetGeom {
    static constexpr int NSTRIP = 3 * VS::Q;         // one time level: 3 cells x Q populations
    static constexpr int NIN = kHistory * NSTRIP;    // input: [strip(t), strip(t-1)]
    // the input tile: NIN values and zeros up to NIN_PAD, a multiple of 32 (the first layer's
    // reduction, K32 products of 32 inputs); NIN_FILL, a multiple of 16, of them come from the
    // strips' normalisation, the rest are zeroed separately
    static constexpr int NIN_PAD = (NIN + 31) / 32 * 32;
    static constexpr int NIN_FILL = (NIN + 15) / 16 * 16;
    static constexpr int ZW = NIN_PAD > kHidden ? NIN_PAD : kHidden;  // width of the input tile
    static constexpr int K32 = NIN_PAD / 32;
    static constexpr int NOUT = entering_count<VS>();
    static constexpr int OFF_W1 = 0;
    static constexpr int OFF_B1 = OFF_W1 + NIN * kHidden;
    static constexpr int OFF_W2 = OFF_B1 + kHidden;
    static constexpr int OFF_B2 = OFF_W2 + kHidden * kHidden;
    static constexpr int OFF_W3 = OFF_B2 + kHidden;
    static constexpr int OFF_B3 = OFF_W3 + kHidden * NOUT;
    static constexpr int NPARAM = OFF_B3 + NOUT;
    // the matrix-core tiles hold an input of at most 128 values and at most 16 outputs (every set
    // but D3Q27); kernels that run the network assert it
    static constexpr bool fits = NIN_PAD <= 128 && NOUT <= 16;
};

// Per-wave LDS tiles (bfloat16 bits); ZW = width of the input tile, a multiple of 16.  16-byte
// aligned (every member's size is a multiple of 16 bytes): the 32-wide A operands are 16-byte reads.
template <int ZW>
struct alignas(16) WaveTiles {
    unsigned short z[16][ZW];
    unsigned short h1[16][64];
    unsigned short h2[16][64];
    unsigned short dy[16][16];
    unsigned short da2[16][64];
    unsigned short da1[16][64];
};

// Per-wave LDS tiles of the forward pass alone (inference), aligned as WaveTiles.  Each row is
// padded by kTilePad values (16 bytes): with rows of 64 or 128 values every row would start in
// LDS bank 0, and the 16 rows that a wave writes or reads at one column would all hit the same
// banks; with the pad, row r starts 4 r banks further, so 8 consecutive rows cover all 32 banks
// (the operand reads, 16 bytes per lane, are conflict-free; the column writes conflict 2-way).
// The second hidden layer h2 reuses z's storage (z is dead once the first layer has read it;
// ZW >= 64), which leaves room for one more block per CU in the network kernels.
constexpr int kTilePad = 8;
template <int ZW>
struct alignas(16) FwdTiles {
    unsigned short z[16][ZW + kTilePad];
    unsigned short h1[16][64 + kTilePad];
};
template <int ZW>
struct FwdView {
    unsigned short (&z)[16][ZW + kTilePad];
    unsigned short (&h1)[16][64 + kTilePad];
    unsigned short (&h2)[16][64 + kTilePad];
};
template <int ZW>
__device__ inline FwdView<ZW> fwd_view(FwdTiles<ZW> &t) {
    static_assert(ZW >= 64, "h2 fits in z's storage");
    return {t.z, t.h1, *reinterpret_cast<unsigned short (*)[16][64 + kTilePad]>(&t.z[0][0])};
}

// A operand from an LDS tile X[16][LD] (rows = samples): columns kk*16 + 4 (l/16) + e.
template <int LD>
__device__ __forceinline__ bf16x4 a_rows(const unsigned short (*X)[LD], int kk, int lane) {
    const int i = lane & 15, k0 = kk * 16 + 4 * (lane >> 4);
    bf16x4 a;
    a.x = (short)X[i][k0]; a.y = (short)X[i][k0 + 1]; a.z = (short)X[i][k0 + 2]; a.w = (short)X[i][k0 + 3];
    return a;
}
// 32-wide A operand from an LDS tile X[16][LD] (rows = samples): columns kk*32 + 8 (l/16) + e, one
// 16-byte read (LD is a multiple of 8, so every row and every 8-column group is 16-byte aligned).
template <int LD>
__device__ __forceinline__ bf16x8 a_rows32(const unsigned short (*X)[LD], int kk, int lane) {
    static_assert(LD % 8 == 0, "16-byte aligned rows");
    const int i = lane & 15, k0 = kk * 32 + 8 * (lane >> 4);
    bf16x8 a;
    __builtin_memcpy(&a, __builtin_assume_aligned(&X[i][k0], 16), sizeof(a));
    return a;
}
// A operand = transpose of an LDS tile: A[i][k] = X[k][mt*16 + i] (rows of A = tile columns).
template <int LD>
__device__ __forceinline__ bf16x4 a_cols(const unsigned short (*X)[LD], int mt, int lane) {
    const int i = mt * 16 + (lane & 15), k0 = 4 * (lane >> 4);
    bf16x4 a;
    a.x = (short)X[k0][i]; a.y = (short)X[k0 + 1][i]; a.z = (short)X[k0 + 2][i]; a.w = (short)X[k0 + 3][i];
    return a;
}
// B operand from an LDS tile: B[k][j] = X[k][nt*16 + j], k = the 16 samples.
template <int LD>
__device__ __forceinline__ bf16x4 b_rows(const unsigned short (*X)[LD], int nt, int lane) {
    const int j = nt * 16 + (lane & 15), k0 = 4 * (lane >> 4);
    bf16x4 b;
    b.x = (short)X[k0][j]; b.y = (short)X[k0 + 1][j]; b.z = (short)X[k0 + 2][j]; b.w = (short)X[k0 + 3][j];
    return b;
}
// B operand from a row-major FP32 matrix W[rows][cols]: B[k][j] = W[kk*16 + k][nt*16 + j],
// zero outside the matrix.
__device__ __forceinline__ bf16x4 b_weight(const float *__restrict__ W, int rows, int cols, int kk, int nt, int lane) {
    const int j = nt * 16 + (lane & 15), k0 = kk * 16 + 4 * (lane >> 4);
    short v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int k = k0 + e;
        v[e] = (k < rows && j < cols) ? (short)bf16_bits(W[k * cols + j]) : (short)0;
    }
    bf16x4 b = {v[0], v[1], v[2], v[3]};
    return b;
}
// 32-wide B operand from a row-major FP32 matrix: B[k][j] = W[kk*32 + k][nt*16 + j], zero outside.
__device__ __forceinline__ bf16x8 b_weight32(const float *__restrict__ W, int rows, int cols, int kk, int nt, int lane) {
    const int j = nt * 16 + (lane & 15), k0 = kk * 32 + 8 * (lane >> 4);
    bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        b[e] = (k < rows && j < cols) ? (short)bf16_bits(W[k * cols + j]) : (short)0;
    }
    return b;
}
// B operand from the transpose of W[rows][cols]: B[k][j] = W[nt*16 + j][kk*16 + k].
__device__ __forceinline__ bf16x4 b_weight_t(const float *__restrict__ W, int rows, int cols, int kk, int nt, int lane) {
    const int j = nt * 16 + (lane & 15), k0 = kk * 16 + 4 * (lane >> 4);
    short v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int k = k0 + e;
        v[e] = (j < rows && k < cols) ? (short)bf16_bits(W[j * cols + k]) : (short)0;
    }
    bf16x4 b = {v[0], v[1], v[2], v[3]};
    return b;
}

// Forward pass of one tile: z (already in LDS) -> h1, h2 (LDS) and y (C layout, 16 x 16).
template <class VS, class TT>
__device__ floatx4 net_forward_tile(const float *__restrict__ P, TT &T, int lane) {
    using G = NetGeom<VS>;
    const int row0 = 4 * (lane >> 4), col = lane & 15;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        floatx4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < G::K32; ++kk)
            acc = mfma32(a_rows32(T.z, kk, lane), b_weight32(P + G::OFF_W1, G::NIN, kHidden, kk, nt, lane), acc);
        const float bias = P[G::OFF_B1 + nt * 16 + col];
#pragma unroll
        for (int e = 0; e < 4; ++e) T.h1[row0 + e][nt * 16 + col] = bf16_bits(fmaxf(acc[e] + bias, 0.0f));
    }
    wave_lds_sync();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        floatx4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
            acc = mfma32(a_rows32(T.h1, kk, lane), b_weight32(P + G::OFF_W2, kHidden, kHidden, kk, nt, lane), acc);
        const float bias = P[G::OFF_B2 + nt * 16 + col];
#pragma unroll
        for (int e = 0; e < 4; ++e) T.h2[row0 + e][nt * 16 + col] = bf16_bits(fmaxf(acc[e] + bias, 0.0f));
    }
    wave_lds_sync();
    floatx4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
        acc = mfma32(a_rows32(T.h2, kk, lane), b_weight32(P + G::OFF_W3, kHidden, G::NOUT, kk, 0, lane), acc);
    const float bias = col < G::NOUT ? P[G::OFF_B3 + col] : 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] += bias;
    return acc;
}

// The forward pass's weights as bfloat16 B-operand fragments (one 16-byte LDS read per lane and
// product) and its FP32 biases, staged once per block.
template <class VS>
struct NetFrags {
    bf16x8 w1[NetGeom<VS>::K32][4][64];
    bf16x8 w2[2][4][64];
    bf16x8 w3[2][64];
    float b1[kHidden], b2[kHidden], b3[16];
};

// Every thread of a 256-thread block must call this (it ends with a block barrier).  Fragment
// (kk, nt, l) of a matrix is handled by thread 64 nt + l for every kk, so each thread's work is
// fixed at compile time: all its global loads are issued before the first conversion, and the
// staging costs about one memory latency.
template <class VS>
__device__ void stage_forward_weights(const float *__restrict__ P, NetFrags<VS> &F) {
    using G = NetGeom<VS>;
    constexpr int K32 = G::K32;
    const int tid = threadIdx.x, l = tid & 63, nt = (tid >> 6) & 3;
    const int j = nt * 16 + (l & 15), r8 = 8 * (l >> 4);
    float v1[K32][8], v2[2][8], v3[8];
#pragma unroll
    for (int kk = 0; kk < K32; ++kk)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = kk * 32 + r8 + e;
            v1[kk][e] = k < G::NIN ? P[G::OFF_W1 + k * kHidden + j] : 0.0f;
        }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int e = 0; e < 8; ++e) v2[kk][e] = P[G::OFF_W2 + (kk * 32 + r8 + e) * kHidden + j];
    // W3 has one column tile and two k-blocks: thread 64 nt + l takes k-block nt & 1 (stored by
    // the threads with nt < 2)
    const int j3 = l & 15;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = (nt & 1) * 32 + r8 + e;
        v3[e] = j3 < G::NOUT ? P[G::OFF_W3 + k * G::NOUT + j3] : 0.0f;
    }
    float bias = 0.0f;
    if (tid < kHidden)
        bias = P[G::OFF_B1 + tid];
    else if (tid < 2 * kHidden)
        bias = P[G::OFF_B2 + tid - kHidden];
    else if (tid < 2 * kHidden + 16)
        bias = tid - 2 * kHidden < G::NOUT ? P[G::OFF_B3 + tid - 2 * kHidden] : 0.0f;
    auto pack8 = [](const float (&v)[8]) {
        bf16x8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e) b[e] = (short)bf16_bits(v[e]);
        return b;
    };
#pragma unroll
    for (int kk = 0; kk < K32; ++kk) F.w1[kk][nt][l] = pack8(v1[kk]);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) F.w2[kk][nt][l] = pack8(v2[kk]);
    if (nt < 2) F.w3[nt][l] = pack8(v3);
    if (tid < kHidden)
        F.b1[tid] = bias;
    else if (tid < 2 * kHidden)
        F.b2[tid - kHidden] = bias;
    else if (tid < 2 * kHidden + 16)
        F.b3[tid - 2 * kHidden] = bias;
    __syncthreads();
}

// net_forward_tile with the staged weights: the same products and roundings.
template <class VS, class TT>
__device__ floatx4 net_forward_tile_staged(const NetFrags<VS> &F, TT &T, int lane) {
    using G = NetGeom<VS>;
    const int row0 = 4 * (lane >> 4), col = lane & 15;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        floatx4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < G::K32; ++kk) acc = mfma32(a_rows32(T.z, kk, lane), F.w1[kk][nt][lane], acc);
        const float bias = F.b1[nt * 16 + col];
#pragma unroll
        for (int e = 0; e < 4; ++e) T.h1[row0 + e][nt * 16 + col] = bf16_bits(fmaxf(acc[e] + bias, 0.0f));
    }
    wave_lds_sync();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        floatx4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) acc = mfma32(a_rows32(T.h1, kk, lane), F.w2[kk][nt][lane], acc);
        const float bias = F.b2[nt * 16 + col];
#pragma unroll
        for (int e = 0; e < 4; ++e) T.h2[row0 + e][nt * 16 + col] = bf16_bits(fmaxf(acc[e] + bias, 0.0f));
    }
    wave_lds_sync();
    floatx4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) acc = mfma32(a_rows32(T.h2, kk, lane), F.w3[kk][lane], acc);
    const float bias = F.b3[col];
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[e] += bias;
    return acc;
}

// Values of a tile per lane: v = g + 4 t (t < tile_vals) of row lane & 15, g = lane >> 4.
template <class VS>
constexpr int tile_vals() {
    return (NetGeom<VS>::NIN_FILL + 3) / 4;
}

// Normalise a tile whose values are already in registers (vals, zero for rows >= nrows and
// v >= n_in) into T.z as bf16 of x / rms(x); returns rms of row (lane & 15) in every lane that
// holds that row.  With EW (v -> weight, 0 for most inputs), also returns in *m_out the row's
// max |x| and in *e_out sum_v EW(v) (x_v / max|x|)^2 (an energy in units of the row's max, no
// underflow).  A row whose max is below 2^-100 is scaled by 2^64 first (exact), so the
// reciprocals of its max and rms cannot overflow; the returned max and rms are scaled back.
template <class VS, class TT, class EWFn>
__device__ float normalise_tile(TT &T, int lane, float (&vals)[tile_vals<VS>()], EWFn EW, float *m_out, float *e_out) {
    using G = NetGeom<VS>;
    const int r = lane & 15, g = lane >> 4;
    float m = 0.0f;
#pragma unroll
    for (int t = 0; t < tile_vals<VS>(); ++t) m = fmaxf(m, fabsf(vals[t]));
    m = fmaxf(m, __shfl_xor(m, 16, 64));
    m = fmaxf(m, __shfl_xor(m, 32, 64));
    const float pre = m < 0x1p-100f ? 0x1p64f : 1.0f;
    m *= pre;
    const float im = m > 0.0f ? 1.0f / m : 0.0f;
    float ss = 0.0f, ee = 0.0f;
#pragma unroll
    for (int t = 0; t < tile_vals<VS>(); ++t) {
        vals[t] *= pre;
        const float q = vals[t] * im;
        ss += q * q;
        const int v = g + 4 * t;
        if (v < G::NIN) ee += EW(v) * q * q;
    }
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    ee += __shfl_xor(ee, 16, 64);
    ee += __shfl_xor(ee, 32, 64);
    const float s = m * sqrtf(ss / (float)G::NIN);
    const float is = s > 0.0f ? 1.0f / s : 0.0f;
#pragma unroll
    for (int t = 0; t < tile_vals<VS>(); ++t) {
        const int v = g + 4 * t;
        if (v < G::NIN_FILL) T.z[r][v] = v < G::NIN ? bf16_bits(vals[t] * is) : (unsigned short)0;
    }
    // the columns between NIN_FILL and NIN_PAD (another 16 where NIN_FILL is an odd multiple of 16)
#pragma unroll
    for (int t = 0; t < (G::NIN_PAD - G::NIN_FILL) / 4; ++t) T.z[r][G::NIN_FILL + g + 4 * t] = 0;
    wave_lds_sync();
    if (m_out) *m_out = m / pre;
    if (e_out) *e_out = ee;
    return s / pre;
}

// Load a tile of raw strips (rows >= nrows are zero) and normalise it as normalise_tile does.
// X(row, v) gives strip value v; ON(row, v, x) sees every loaded value (row < nrows, v < n_in).
template <class VS, class TT, class LoadFn, class EWFn, class OnFn>
__device__ float load_normalised_tile(TT &T, int nrows, int lane, LoadFn X, EWFn EW, float *m_out, float *e_out,
                                      OnFn ON) {
    using G = NetGeom<VS>;
    const int r = lane & 15, g = lane >> 4;
    float vals[tile_vals<VS>()];
#pragma unroll
    for (int t = 0; t < tile_vals<VS>(); ++t) {
        const int v = g + 4 * t;
        vals[t] = (r < nrows && v < G::NIN) ? X(r, v) : 0.0f;
    }
    // after every load is issued (a store of a loaded value waits for that load)
#pragma unroll
    for (int t = 0; t < tile_vals<VS>(); ++t) {
        const int v = g + 4 * t;
        if (r < nrows && v < G::NIN) ON(r, v, vals[t]);
    }
    return normalise_tile<VS>(T, lane, vals, EW, m_out, e_out);
}
template <class VS, class TT, class LoadFn, class EWFn>
__device__ float load_normalised_tile(TT &T, int nrows, int lane, LoadFn X, EWFn EW, float *m_out, float *e_out) {
    return load_normalised_tile<VS>(T, nrows, lane, X, EW, m_out, e_out, [](int, int, float) {});
}
template <class VS, class TT, class LoadFn>
__device__ float load_normalised_tile(TT &T, int nrows, int lane, LoadFn X) {
    return load_normalised_tile<VS>(T, nrows, lane, X, [](int) { return 0.0f; }, nullptr, nullptr);
}

// ------------------------------------------------------------------ batch inference on strips
template <class VS>
__global__ __launch_bounds__(256) void nrbc_forward_kernel(const float *__restrict__ P, const float *__restrict__ strips,
                                                           long long count, float *__restrict__ out) {
    using G = NetGeom<VS>;
    static_assert(G::fits, "network tiles");
    __shared__ FwdTiles<G::ZW> tiles[4];
    __shared__ NetFrags<VS> F;
    stage_forward_weights<VS>(P, F);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    FwdView<G::ZW> T = fwd_view(tiles[wid]);
    const long long ntiles = (count + 15) / 16;
    for (long long tile = (long long)blockIdx.x * 4 + wid; tile < ntiles; tile += (long long)gridDim.x * 4) {
        const long long base = tile * 16;
        const int nrows = (int)min((long long)16, count - base);
        const float s = load_normalised_tile<VS>(T, nrows, lane,
                                                 [&](int r, int v) { return strips[(base + r) * G::NIN + v]; });
        const floatx4 y = net_forward_tile_staged<VS>(F, T, lane);
        // y[e] is row 4 (l/16) + e, column l % 16; the row's rms lives in lane (row)
        const int col = lane & 15;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 4 * (lane >> 4) + e;
            const float srow = __shfl(s, row, 64);
            if (row < nrows && col < G::NOUT) out[(base + row) * G::NOUT + col] = srow * y[e];
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ loss and gradients
// Each wave accumulates the gradients of its tiles in registers and writes one partial row
// (NPARAM gradient values, then its squared-error sum) to ws[wave]; nrbc_reduce_kernel sums the
// rows in a fixed order.  Targets are raw; they are divided by the strip's rms like the
// prediction.  Loss = mean over samples and outputs of (y - t / s)^2.
//   dy  = 2 (y - t/s) / (count k)                       (bf16)
//   dW3 = h2^T dy,  db3 = 1^T dy,   dh2 = dy W3^T,  da2 = dh2 [h2 > 0]   (bf16)
//   dW2 = h1^T da2, db2 = 1^T da2,  dh1 = da2 W2^T, da1 = dh1 [h1 > 0]   (bf16)
//   dW1 = z^T da1,  db1 = 1^T da1
// Column sums use a product with an all-ones bf16 operand, so they are summed in FP32 exactly
// like the weight gradients.
template <class VS>
__global__ __launch_bounds__(256) void nrbc_grad_kernel(const float *__restrict__ P, const float *__restrict__ strips,
                                                        const float *__restrict__ targets, long long count,
                                                        const unsigned long long *__restrict__ nvalid,
                                                        float *__restrict__ ws) {
    static_assert(NetGeom<VS>::fits, "network tiles");
    using G = NetGeom<VS>;
    constexpr int MT1 = G::NIN_PAD / 16;
    __shared__ WaveTiles<G::ZW> tiles[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    WaveTiles<G::ZW> &T = tiles[wid];
    const int row0 = 4 * (lane >> 4), col = lane & 15;
    const float inv_n = (float)(1.0 / ((double)(*nvalid ? *nvalid : 1ull) * G::NOUT));
    bf16x4 ones;
    ones.x = ones.y = ones.z = ones.w = (short)0x3f80;  // bf16 1.0
    const floatx4 zero = {0, 0, 0, 0};

    floatx4 g1[MT1][4], g2[4][4], g3[4], gb1[4], gb2[4], gb3;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int m = 0; m < MT1; ++m) g1[m][a] = zero;
#pragma unroll
        for (int b = 0; b < 4; ++b) g2[a][b] = zero;
        g3[a] = zero;
        gb1[a] = zero;
        gb2[a] = zero;
    }
    gb3 = zero;
    float sq = 0.0f;

    const long long ntiles = (count + 15) / 16;
    for (long long tile = (long long)blockIdx.x * 4 + wid; tile < ntiles; tile += (long long)gridDim.x * 4) {
        const long long base = tile * 16;
        const int nrows = (int)min((long long)16, count - base);
        const float s = load_normalised_tile<VS>(T, nrows, lane,
                                                 [&](int r, int v) { return strips[(base + r) * G::NIN + v]; });
        const floatx4 y = net_forward_tile<VS>(P, T, lane);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = row0 + e;
            const float srow = __shfl(s, row, 64);
            float d = 0.0f;
            if (row < nrows && col < G::NOUT && srow > 0.0f) {
                const float t = targets[(base + row) * G::NOUT + col] / srow;
                const float diff = y[e] - t;
                sq += diff * diff;
                d = 2.0f * diff * inv_n;
            }
            T.dy[row][col] = bf16_bits(d);
        }
        wave_lds_sync();
        // layer 3
        const bf16x4 bdy = b_rows<16>(T.dy, 0, lane);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) g3[mt] = mfma16(a_cols<64>(T.h2, mt, lane), bdy, g3[mt]);
        gb3 = mfma16(ones, bdy, gb3);
        {
            bf16x4 ady;  // A = dy (rows = samples, k = outputs 0..15)
            const int i = lane & 15, k0 = 4 * (lane >> 4);
            ady.x = (short)T.dy[i][k0]; ady.y = (short)T.dy[i][k0 + 1];
            ady.z = (short)T.dy[i][k0 + 2]; ady.w = (short)T.dy[i][k0 + 3];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const floatx4 dh = mfma16(ady, b_weight_t(P + G::OFF_W3, kHidden, G::NOUT, 0, nt, lane), zero);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = row0 + e, c = nt * 16 + col;
                    T.da2[row][c] = bf16_bits(bf16_val(T.h2[row][c]) > 0.0f ? dh[e] : 0.0f);
                }
            }
        }
        wave_lds_sync();
        // layer 2
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x4 bda = b_rows<64>(T.da2, nt, lane);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) g2[mt][nt] = mfma16(a_cols<64>(T.h1, mt, lane), bda, g2[mt][nt]);
            gb2[nt] = mfma16(ones, bda, gb2[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            floatx4 dh = zero;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                dh = mfma16(a_rows(T.da2, kk, lane), b_weight_t(P + G::OFF_W2, kHidden, kHidden, kk, nt, lane), dh);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = row0 + e, c = nt * 16 + col;
                T.da1[row][c] = bf16_bits(bf16_val(T.h1[row][c]) > 0.0f ? dh[e] : 0.0f);
            }
        }
        wave_lds_sync();
        // layer 1
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const bf16x4 bda = b_rows<64>(T.da1, nt, lane);
#pragma unroll
            for (int mt = 0; mt < MT1; ++mt) g1[mt][nt] = mfma16(a_cols<G::ZW>(T.z, mt, lane), bda, g1[mt][nt]);
            gb1[nt] = mfma16(ones, bda, gb1[nt]);
        }
        wave_lds_sync();
    }
    // partial row of this wave: C layout element (row = 4 (l/16) + e, col = l % 16)
    float *out = ws + (size_t)(blockIdx.x * 4 + wid) * (G::NPARAM + 1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int r = row0 + e;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int c = nt * 16 + col;
#pragma unroll
            for (int mt = 0; mt < MT1; ++mt) {
                const int in = mt * 16 + r;
                if (in < G::NIN) out[G::OFF_W1 + in * kHidden + c] = g1[mt][nt][e];
            }
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) out[G::OFF_W2 + (mt * 16 + r) * kHidden + c] = g2[mt][nt][e];
            if (r == 0) {
                out[G::OFF_B1 + c] = gb1[nt][e];
                out[G::OFF_B2 + c] = gb2[nt][e];
            }
        }
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            if (col < G::NOUT) out[G::OFF_W3 + (mt * 16 + r) * G::NOUT + col] = g3[mt][e];
        if (r == 0 && col < G::NOUT) out[G::OFF_B3 + col] = gb3[e];
    }
    // squared-error sum of the wave (lanes hold disjoint elements)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if (lane == 0) out[G::NPARAM] = sq;
}

[[maybe_unused]] static __global__ void nrbc_zero_counter(unsigned long long *c) { *c = 0ull; }

// Number of strips with at least one non-zero value (the samples the loss averages over).
template <class VS>
__global__ __launch_bounds__(256) void nrbc_count_valid(const float *__restrict__ strips, long long count,
                                                        unsigned long long *__restrict__ out) {
    using G = NetGeom<VS>;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    bool nz = false;
    if (t < count)
        for (int v = 0; v < G::NIN; ++v) nz = nz || strips[t * G::NIN + v] != 0.0f;
    const unsigned long long b = __ballot(nz);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(out, (unsigned long long)__popcll(b));
}

// grad[p] = sum over waves of ws[w][p] (fixed order); loss = sum of the squared errors / (count k).
[[maybe_unused]] static __global__ __launch_bounds__(256) void nrbc_reduce_kernel(const float *__restrict__ ws, int nwaves, int nparam,
                                                          const unsigned long long *__restrict__ nvalid, int nout,
                                                          float *__restrict__ grad, float *__restrict__ loss) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > nparam) return;
    double acc = 0.0;
    for (int w = 0; w < nwaves; ++w) acc += (double)ws[(size_t)w * (nparam + 1) + p];
    if (p < nparam)
        grad[p] = (float)acc;
    else if (loss)
        *loss = *nvalid ? (float)(acc / ((double)*nvalid * nout)) : 0.0f;
}

// Adam (Kingma & Ba) on FP32 master parameters; t counts from 1.
[[maybe_unused]] static __global__ __launch_bounds__(256) void nrbc_adam_kernel(long long n, float *__restrict__ P, const float *__restrict__ g,
                                                        float *__restrict__ m, float *__restrict__ v, float lr,
                                                        float b1, float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace lbm
