// Learned initial guess for the Krylov solve: per-(wire, incidence) features,
// a 192-128-128-128-14 SiLU network on BF16 matrix cores with FP32
// accumulation (forward, backward, Adam), and the maps between solved
// currents and network outputs.  Not part of the paper's method: the solver
// still drives the true residual of the S-NFC system (eq. 9) to the same
// tolerance, so the guess can only change how many iterations that takes.
//
// Products use v_mfma_f32_16x16x32_bf16: a wave multiplies a 16 x 32 BF16
// tile of A (rows = samples) by a 32 x 16 tile of B into a 16 x 16 FP32
// accumulator.  Each lane supplies 8 consecutive k of one row of A and of
// one column of B (A and B stored k-contiguous), and receives 4 consecutive
// rows of one output column.  Every intermediate of the backward pass is
// written in the layout its consumer needs (row-major for the next data
// product, transposed for the weight-gradient product), so no product reads
// strided memory.
#include <algorithm>

#include "common.hpp"
#include "precond.hpp"
#include "prof.hpp"

namespace chaff {
namespace {

constexpr int KNB = 16, FOWN = 16, FNB = 11, NF = FOWN + KNB * FNB, NH = 128, NO = 14;
constexpr int OW1 = 0, OB1 = OW1 + NF * NH, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH * NH, OW4 = OB3 + NH, OB4 = OW4 + NH * NO, NPARAM = OB4 + NO;
static_assert(NF == CHAFF_MLP_NFEAT && NH == CHAFF_MLP_HIDDEN && NO == CHAFF_MLP_NOUT, "header sizes");
static_assert(NPARAM == CHAFF_MLP_NPARAM, "parameter count");
constexpr int NOP = 16;          // output columns padded to one MFMA tile
constexpr int DYLD = 32;         // row stride of dL/dy (K of the first backward product)
constexpr int ROWS_WG = 128;     // rows per workgroup in the row-parallel products
constexpr int SPLIT_ROWS = 512;  // rows per partial sum of the weight gradients
constexpr double X_SCALE = 0.5;  // network outputs are current departures / 0.5
constexpr int NB_W = 7;          // rooftop unknowns per wire (8 segments)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // nearest even on the FP32 pattern
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// the same rounding (nearest even) by the hardware conversion, for activations
__device__ __forceinline__ uint16_t f2bf_hw(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint16_t d2bf(double x) { return f2bf((float)x); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(p));
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0)); }

// acc[mt][nt] += A rows ap[mt] (k-contiguous, nullptr = zero row) x B rows bp[nt], k in [k0, k1).
template <int MT, int NT>
__device__ __forceinline__ void mma_rows(const uint16_t* const (&ap)[MT], const uint16_t* const (&bp)[NT],
                                         int64_t k0, int64_t k1, f32x4 (&acc)[MT][NT]) {
    const int kb = ((threadIdx.x & 63) >> 4) * 8;
    for (int64_t k = k0; k < k1; k += 32) {
        bf16x8 a[MT], b[NT];
#pragma unroll
        for (int i = 0; i < MT; ++i) a[i] = ap[i] ? ld8(ap[i] + k + kb) : zero8();
#pragma unroll
        for (int j = 0; j < NT; ++j) b[j] = ld8(bp[j] + k + kb);
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
}

// logistic function with the hardware exponential and reciprocal (about 1 ulp each;
// the result is rounded to BF16 or enters a BF16 product)
__device__ __forceinline__ float sigmoidf(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float wave_sum(float v) {  // fixed butterfly order
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------------ parameters -> BF16 operands
// Wt_l [n_out_pad][n_in]  (B operand of the forward product)
// Wn_l [n_in][n_out_pad'] (B operand of the backward data product), l = 2..4
struct Packed {
    uint16_t *wt1, *wt2, *wt3, *wt4, *wn2, *wn3, *wn4;
};

__global__ void k_pack(const float* __restrict__ th, Packed pk) {
    const int which = blockIdx.y;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // (dst, offset of W, n_in, n_out, transposed?, padded width)
    uint16_t* dst;
    int off, nin, nout, pad;
    bool tr;
    switch (which) {
        case 0: dst = pk.wt1; off = OW1; nin = NF; nout = NH; tr = true; pad = NH; break;
        case 1: dst = pk.wt2; off = OW2; nin = NH; nout = NH; tr = true; pad = NH; break;
        case 2: dst = pk.wt3; off = OW3; nin = NH; nout = NH; tr = true; pad = NH; break;
        case 3: dst = pk.wt4; off = OW4; nin = NH; nout = NO; tr = true; pad = NOP; break;
        case 4: dst = pk.wn2; off = OW2; nin = NH; nout = NH; tr = false; pad = NH; break;
        case 5: dst = pk.wn3; off = OW3; nin = NH; nout = NH; tr = false; pad = NH; break;
        default: dst = pk.wn4; off = OW4; nin = NH; nout = NO; tr = false; pad = DYLD; break;
    }
    if (t >= (int64_t)nin * pad) return;
    int i, o;
    if (tr) { o = (int)(t / nin); i = (int)(t % nin); }
    else { i = (int)(t / pad); o = (int)(t % pad); }
    dst[t] = o < nout ? f2bf(th[off + i * nout + o]) : (uint16_t)0;
}

// ------------------------------------------------------------------ forward layers
struct FwdArgs {
    const uint16_t* A;      // [*][lda] BF16 layer input (row m at idx[m] for the first layer)
    int lda;
    const int64_t* a_idx;   // optional row gather of A (first layer)
    const int64_t* t_idx;   // optional row gather of the targets
    int64_t M, Mpad;        // valid rows, padded rows
    const uint16_t* Wt;     // [N][K]
    int K;
    const float* bias;
    // hidden layers
    uint16_t* a_out;        // [Mpad][128] BF16 SiLU(z)
    float* z_out;           // [Mpad][128] FP32 pre-activation (training)
    uint16_t* aT_out;       // [128][Mpad] BF16 SiLU(z) transposed (training)
    // output layer
    float* Y;               // [M][14] (inference)
    const float* T;         // [*][14] targets (training)
    uint16_t* dY;           // [Mpad][32] BF16 2 (y - t) (training)
    uint16_t* dYT;          // [16][Mpad]
    float* loss_part;       // [Mpad/32] per-wave sums of (y - t)^2
};

template <bool LAST, bool TRAIN>
__global__ __launch_bounds__(256) void k_fwd(FwdArgs g) {
    constexpr int NT = LAST ? 1 : NH / 16;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t m0 = wave * 32;
    const uint16_t* ap[2];
    const uint16_t* bp[NT];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int64_t m = m0 + 16 * i + (lane & 15);
        const int64_t src = m < g.M ? (g.a_idx ? g.a_idx[m] : m) : -1;
        ap[i] = src >= 0 ? g.A + src * g.lda : nullptr;
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) bp[j] = g.Wt + (int64_t)(16 * j + (lane & 15)) * g.K;
    f32x4 acc[2][NT];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    mma_rows<2, NT>(ap, bp, 0, g.K, acc);

    const int col = lane & 15;
    const int rq = (lane >> 4) * 4;
    if constexpr (!LAST) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const int n = 16 * j + col;
                const float b = g.bias[n];
                const int64_t mb = m0 + 16 * i + rq;
                uint16_t h[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[i][j][r] + b;
                    h[r] = f2bf(z * sigmoidf(z));
                    g.a_out[(mb + r) * NH + n] = h[r];
                    if (TRAIN) g.z_out[(mb + r) * NH + n] = z;
                }
                if (TRAIN)
                    *reinterpret_cast<uint2*>(g.aT_out + (int64_t)n * g.Mpad + mb) =
                        make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
            }
    } else {
        const float b = col < NO ? g.bias[col] : 0.f;
        float sq = 0.f;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t mb = m0 + 16 * i + rq;
            uint16_t h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t m = mb + r;
                const float y = acc[i][0][r] + b;
                if (!TRAIN) {
                    if (m < g.M && col < NO) g.Y[m * NO + col] = y;
                } else {
                    float d = 0.f;
                    if (m < g.M && col < NO) d = y - g.T[(g.t_idx ? g.t_idx[m] : m) * NO + col];
                    sq += d * d;
                    h[r] = f2bf(2.0f * d);
                    g.dY[m * DYLD + col] = h[r];
                    g.dY[m * DYLD + NOP + col] = 0;
                }
            }
            if (TRAIN)
                *reinterpret_cast<uint2*>(g.dYT + (int64_t)col * g.Mpad + mb) =
                    make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
        }
        if (TRAIN) {
            sq = wave_sum(sq);
            if (lane == 0) g.loss_part[wave] = sq;
        }
    }
}

// ------------------------------------------------------------------ fused inference
// All four layers in one persistent kernel: each workgroup copies the BF16
// weights into LDS once (rows padded by 8 elements so that the 16 rows a
// ds_read_b128 touches fall in distinct banks), then every wave walks its own
// 32-row tiles: layer 1 reads the features from HBM, the hidden activations
// stay in the wave's LDS tile, and only the 14 outputs are written.  Weight
// traffic is 116 KB per workgroup instead of per 32-row tile.
constexpr int FLD1 = NF + 8, FLDH = NH + 8;   // padded LDS row strides (BF16)
constexpr int FUSED_LDS = (NH * FLD1 + 2 * NH * FLDH + NOP * FLDH + 4 * 32 * FLDH) * 2;

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(256) void k_fwd_fused(const uint16_t* __restrict__ feat, int64_t M,
                                                   const float* __restrict__ th, Packed pk, float* __restrict__ Y) {
    extern __shared__ uint16_t lds[];
    uint16_t* w1 = lds;                      // [128][FLD1]
    uint16_t* w2 = w1 + NH * FLD1;           // [128][FLDH]
    uint16_t* w3 = w2 + NH * FLDH;           // [128][FLDH]
    uint16_t* w4 = w3 + NH * FLDH;           // [16][FLDH]
    uint16_t* act = w4 + NOP * FLDH;         // [4 waves][32][FLDH]
    // weights -> LDS (16-byte chunks)
    for (int t = threadIdx.x; t < NH * (NF / 8); t += 256) {
        const int r = t / (NF / 8), c = (t % (NF / 8)) * 8;
        *reinterpret_cast<uint4*>(w1 + r * FLD1 + c) = *reinterpret_cast<const uint4*>(pk.wt1 + r * NF + c);
    }
    for (int t = threadIdx.x; t < NH * (NH / 8); t += 256) {
        const int r = t / (NH / 8), c = (t % (NH / 8)) * 8;
        *reinterpret_cast<uint4*>(w2 + r * FLDH + c) = *reinterpret_cast<const uint4*>(pk.wt2 + r * NH + c);
        *reinterpret_cast<uint4*>(w3 + r * FLDH + c) = *reinterpret_cast<const uint4*>(pk.wt3 + r * NH + c);
    }
    for (int t = threadIdx.x; t < NOP * (NH / 8); t += 256) {
        const int r = t / (NH / 8), c = (t % (NH / 8)) * 8;
        *reinterpret_cast<uint4*>(w4 + r * FLDH + c) = *reinterpret_cast<const uint4*>(pk.wt4 + r * NH + c);
    }
    __syncthreads();
    // The weights are the A operand (rows = output features) and the activations
    // the B operand (columns = sample rows): a lane then holds 4 consecutive
    // output features of one sample, written to the LDS tile as one 8-byte store.
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t* my = act + w * 32 * FLDH;
    const int l16 = lane & 15, g4 = (lane >> 4) * 4, kb = (lane >> 4) * 8;
    const int64_t n_tiles = (M + 31) / 32;
    constexpr int KS1 = NF / 32, MT = NH / 16;
    auto load_tile = [&](int64_t tile, bf16x8 (&fa)[KS1][2]) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t m = tile * 32 + 16 * j + l16;
#pragma unroll
            for (int ks = 0; ks < KS1; ++ks) fa[ks][j] = m < M ? ld8(feat + m * NF + ks * 32 + kb) : zero8();
        }
    };
    // bias + SiLU of acc -> BF16 activation tile
    auto to_tile = [&](const f32x4 (&acc)[MT][2], const float* bias) {
        wave_lds_sync();
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int f0 = 16 * i + g4;
            const float4 b = *reinterpret_cast<const float4*>(bias + f0);
            const float bb[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                uint16_t h[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float z = acc[i][j][r] + bb[r];
                    h[r] = f2bf_hw(z * sigmoidf(z));
                }
                *reinterpret_cast<uint2*>(my + (16 * j + l16) * FLDH + f0) =
                    make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
            }
        }
        wave_lds_sync();
    };
    const int64_t t_step = (int64_t)gridDim.x * 4;
    int64_t tile = (int64_t)blockIdx.x * 4 + w;
    bf16x8 fa[KS1][2];
    if (tile < n_tiles) load_tile(tile, fa);
    for (; tile < n_tiles; tile += t_step) {
        const int64_t m0 = tile * 32;
        bf16x8 fnext[KS1][2];
        if (tile + t_step < n_tiles) load_tile(tile + t_step, fnext);
        f32x4 acc[MT][2];
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) {   // layer 1
#pragma unroll
            for (int i = 0; i < MT; ++i) {
                const bf16x8 a = ld8(w1 + (16 * i + l16) * FLD1 + ks * 32 + kb);
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, fa[ks][j], acc[i][j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {   // layers 2 and 3
            to_tile(acc, th + (layer == 0 ? OB1 : OB2));
            const uint16_t* wl = layer == 0 ? w2 : w3;
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
            for (int k = 0; k < NH; k += 32) {
                bf16x8 b[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = ld8(my + (16 * j + l16) * FLDH + k + kb);
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const bf16x8 a = ld8(wl + (16 * i + l16) * FLDH + k + kb);
#pragma unroll
                    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
                }
            }
        }
        to_tile(acc, th + OB3);
        f32x4 out[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
        for (int k = 0; k < NH; k += 32) {   // output layer (14 of 16 rows of W4^T used)
            const bf16x8 a = ld8(w4 + l16 * FLDH + k + kb);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                out[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, ld8(my + (16 * j + l16) * FLDH + k + kb), out[j], 0, 0, 0);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t m = m0 + 16 * j + l16;
            if (m < M) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int f = g4 + r;
                    if (f < NO) Y[m * NO + f] = out[j][r] + th[OB4 + f];
                }
            }
        }
#pragma unroll
        for (int ks = 0; ks < KS1; ++ks) {
            fa[ks][0] = fnext[ks][0];
            fa[ks][1] = fnext[ks][1];
        }
    }
}

// ------------------------------------------------------------------ backward
// dZ_prev = (dZ W^T) * SiLU'(z_prev): A = dZ [Mpad][lda], B = Wn [128][K].
struct BwdArgs {
    const uint16_t* dZ;
    int lda, K;
    int64_t Mpad;
    const uint16_t* Wn;
    const float* z_prev;     // [Mpad][128]
    uint16_t* dZ_out;        // [Mpad][128] or nullptr
    uint16_t* dZT_out;       // [128][Mpad]
};

__global__ __launch_bounds__(256) void k_bwd(BwdArgs g) {
    constexpr int NT = NH / 16;
    const int lane = threadIdx.x & 63;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32;
    const uint16_t* ap[2];
    const uint16_t* bp[NT];
#pragma unroll
    for (int i = 0; i < 2; ++i) ap[i] = g.dZ + (m0 + 16 * i + (lane & 15)) * g.lda;
#pragma unroll
    for (int j = 0; j < NT; ++j) bp[j] = g.Wn + (int64_t)(16 * j + (lane & 15)) * g.K;
    f32x4 acc[2][NT];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    mma_rows<2, NT>(ap, bp, 0, g.K, acc);
    const int col = lane & 15;
    const int rq = (lane >> 4) * 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int n = 16 * j + col;
            const int64_t mb = m0 + 16 * i + rq;
            uint16_t h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float z = g.z_prev[(mb + r) * NH + n];
                const float s = sigmoidf(z);
                h[r] = f2bf(acc[i][j][r] * (s * (1.0f + z * (1.0f - s))));
                if (g.dZ_out) g.dZ_out[(mb + r) * NH + n] = h[r];
            }
            *reinterpret_cast<uint2*>(g.dZT_out + (int64_t)n * g.Mpad + mb) =
                make_uint2(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16));
        }
}

// Partial weight gradients over one split of SPLIT_ROWS rows:
// part[s][w_off + i*n_out + o] = sum_m aT[i][m] dZT[o][m].
template <int NT>
__global__ __launch_bounds__(64) void k_wgrad(const uint16_t* __restrict__ aT, const uint16_t* __restrict__ dZT,
                                              int64_t Mpad, int n_out, int w_off, float* __restrict__ part) {
    const int lane = threadIdx.x;
    const int i0 = blockIdx.x * 16, o0 = blockIdx.y * 16 * NT;
    const int64_t s = blockIdx.z;
    const uint16_t* ap[1] = {aT + (int64_t)(i0 + (lane & 15)) * Mpad};
    const uint16_t* bp[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) bp[j] = dZT + (int64_t)(o0 + 16 * j + (lane & 15)) * Mpad;
    f32x4 acc[1][NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[0][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    mma_rows<1, NT>(ap, bp, s * SPLIT_ROWS, (s + 1) * SPLIT_ROWS, acc);
    float* dst = part + s * NPARAM + w_off;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int o = o0 + 16 * j + (lane & 15);
        if (o >= n_out) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[(int64_t)(i0 + (lane >> 4) * 4 + r) * n_out + o] = acc[0][j][r];
    }
}

// Partial bias gradients: one wave per (output unit, split).
__global__ __launch_bounds__(64) void k_bgrad(const uint16_t* __restrict__ dYT, const uint16_t* __restrict__ dZT3,
                                              const uint16_t* __restrict__ dZT2, const uint16_t* __restrict__ dZT1,
                                              int64_t Mpad, float* __restrict__ part) {
    const int u = blockIdx.x;  // 0..13: b4, then b3, b2, b1 (128 each)
    const int64_t s = blockIdx.y;
    const uint16_t* row;
    int off;
    if (u < NO) { row = dYT + (int64_t)u * Mpad; off = OB4 + u; }
    else if (u < NO + NH) { row = dZT3 + (int64_t)(u - NO) * Mpad; off = OB3 + (u - NO); }
    else if (u < NO + 2 * NH) { row = dZT2 + (int64_t)(u - NO - NH) * Mpad; off = OB2 + (u - NO - NH); }
    else { row = dZT1 + (int64_t)(u - NO - 2 * NH) * Mpad; off = OB1 + (u - NO - 2 * NH); }
    row += s * SPLIT_ROWS;
    float v = 0.f;
    for (int k = threadIdx.x; k < SPLIT_ROWS; k += 64) v += bf2f(row[k]);
    v = wave_sum(v);
    if (threadIdx.x == 0) part[s * NPARAM + off] = v;
}

// grad = scale * sum over splits (fixed order); the last block also reduces the loss.
__global__ void k_reduce(const float* __restrict__ part, int64_t nsplit, float scale, float* __restrict__ grad,
                         const float* __restrict__ loss_part, int64_t nloss, float* __restrict__ loss) {
    if (blockIdx.x == gridDim.x - 1) {
        if (threadIdx.x == 0 && loss) {
            double acc = 0.0;
            for (int64_t i = 0; i < nloss; ++i) acc += loss_part[i];
            *loss = (float)(acc * (double)scale);
        }
        return;
    }
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NPARAM) return;
    float acc = 0.f;
    for (int64_t s = 0; s < nsplit; ++s) acc += part[s * NPARAM + j];
    grad[j] = acc * scale;
}

// Input features transposed (and gathered): fT[f][m] = feat[idx[m]][f], zero for m >= M.
__global__ __launch_bounds__(256) void k_feat_t(const uint16_t* __restrict__ feat, const int64_t* __restrict__ idx,
                                                int64_t M, int64_t Mpad, uint16_t* __restrict__ fT) {
    __shared__ uint16_t tile[64][NF + 2];
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    for (int t = threadIdx.x; t < 64 * NF; t += 256) {
        const int r = t / NF, f = t % NF;
        const int64_t m = m0 + r;
        tile[r][f] = m < M ? feat[(idx ? idx[m] : m) * NF + f] : (uint16_t)0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * NF; t += 256) {
        const int f = t / 64, r = t % 64;
        fT[(int64_t)f * Mpad + m0 + r] = tile[r][f];
    }
}

__global__ void k_adam(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= NPARAM) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.0f - b1) * gj;
    const float vj = b2 * v[j] + (1.0f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    th[j] -= lr * (mj / bc1) / (sqrtf(vj / bc2) + eps);
}

// ------------------------------------------------------------------ features
// FP64 squared centroid distance ((dx*dx + dy*dy) + dz*dz), every operation
// rounded on its own, as in the near-set test.
__device__ __forceinline__ double dist2(const Wire& a, const Wire& b) {
#pragma clang fp contract(off)
    const double dx = b.cx - a.cx, dy = b.cy - a.cy, dz = b.cz - a.cz;
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    double s = xx + yy;
    s = s + zz;
    return s;
}

__device__ __forceinline__ double sinc_d(double x) {
    if (fabs(x) < 1e-4) return 1.0 - x * x / 6.0;
    return sin(x) / x;
}

constexpr int FW_CAND = 256;   // near-set rows up to this length are ranked in parallel

// One wave per wire p (caller order) and the rows p*R + r of it that fall in
// the requested range.  The 16 nearest neighbours are chosen once per wire:
// every lane ranks its candidates by counting the candidates with a smaller
// (squared distance, caller index) key (rows longer than FW_CAND fall back to
// repeated minimum search), and the neighbours' geometry is staged in LDS.
// The features that do not depend on the incidence are formed once per wire.
__global__ __launch_bounds__(64) void k_features(const Wire* __restrict__ wires, const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ iperm,
                                                 const int64_t* __restrict__ row_ptr,
                                                 const int32_t* __restrict__ col_idx, int64_t R, int64_t row0,
                                                 int64_t n_rows, const double* __restrict__ k_hat,
                                                 const double* __restrict__ e_hat, double k, double lam, double d_c,
                                                 uint16_t* __restrict__ feat) {
#pragma clang fp contract(off)
    __shared__ double cd2[FW_CAND];
    __shared__ int32_t cid[FW_CAND], cint[FW_CAND];
    __shared__ int32_t slot[KNB];
    __shared__ double sg[KNB][8];   // d.x, d.y, d.z, d2, t'.x, t'.y, t'.z, L'
    __shared__ uint16_t fixed[KNB][4];   // |d|/d_c, length feature, Re, Im exp(-j k |d|)
    const int lane = threadIdx.x;
    const int64_t p = row0 / R + blockIdx.x;
    const int64_t rb = p * R > row0 ? p * R : row0;
    const int64_t re = (p + 1) * R < row0 + n_rows ? (p + 1) * R : row0 + n_rows;
    if (rb >= re) return;   // uniform over the (single-wave) block
    const int32_t ip = iperm[p];
    const Wire w = wires[ip];
    const int64_t e0 = row_ptr[ip], e1 = row_ptr[ip + 1];
    const int64_t ne = e1 - e0;   // includes the diagonal
    const int64_t cnt = ne - 1;
    if (lane < KNB) slot[lane] = -1;
    if (ne <= FW_CAND) {
        for (int64_t t = lane; t < ne; t += 64) {
            const int32_t c = col_idx[e0 + t];
            cint[t] = c;
            cid[t] = perm[c];
            cd2[t] = c == ip ? 0.0 : dist2(w, wires[c]);
        }
        __syncthreads();
        for (int64_t t = lane; t < ne; t += 64) {
            if (cint[t] == ip) continue;
            const double d2 = cd2[t];
            const int32_t id = cid[t];
            int rank = 0;
            for (int64_t u = 0; u < ne; ++u) {
                if (cint[u] == ip) continue;
                const double du = cd2[u];
                rank += (du < d2 || (du == d2 && cid[u] < id)) ? 1 : 0;
            }
            if (rank < KNB) slot[rank] = cint[t];
        }
    } else {   // long row: repeated minimum search (the same on every lane)
        double pd2 = -1.0;
        int32_t pid = -1;
        for (int j = 0; j < KNB; ++j) {
            double bd2 = INFINITY;
            int32_t bid = INT32_MAX, bint = -1;
            for (int64_t e = e0; e < e1; ++e) {
                const int32_t c = col_idx[e];
                if (c == ip) continue;
                const double d2 = dist2(w, wires[c]);
                const int32_t id = perm[c];
                const bool after = d2 > pd2 || (d2 == pd2 && id > pid);
                const bool before = d2 < bd2 || (d2 == bd2 && id < bid);
                if (after && before) { bd2 = d2; bid = id; bint = c; }
            }
            if (bint < 0) break;
            if (lane == 0) slot[j] = bint;
            pd2 = bd2;
            pid = bid;
        }
    }
    __syncthreads();
    // per-slot geometry and the incidence-independent features
    if (lane < KNB && slot[lane] >= 0) {
        const Wire v = wires[slot[lane]];
        const double d2 = dist2(w, v);
        sg[lane][0] = v.cx - w.cx;
        sg[lane][1] = v.cy - w.cy;
        sg[lane][2] = v.cz - w.cz;
        sg[lane][3] = d2;
        sg[lane][4] = v.tx;
        sg[lane][5] = v.ty;
        sg[lane][6] = v.tz;
        sg[lane][7] = v.len;
        double sn, cs;
        sincos(k * sqrt(d2), &sn, &cs);
        fixed[lane][0] = d2bf(sqrt(d2) / d_c);
        fixed[lane][1] = d2bf(10.0 * (v.len / lam - 0.5));
        fixed[lane][2] = d2bf(cs);
        fixed[lane][3] = d2bf(-sn);
    }
    __syncthreads();
    // two rows per pass: lanes 0-31 the first, 32-63 the second; within a half,
    // lane m < 16 writes neighbour slot m, 16 <= m < 23 own rooftop m - 16,
    // m = 23 the two scalar own features.  Every active lane evaluates exactly
    // one sine/cosine per row.
    const double D = w.len / 8.0;
    const int half = lane >> 5, m = lane & 31;
    for (int64_t row2 = rb; row2 < re; row2 += 2) {
        const int64_t row = row2 + half;
        const bool live = row < re;
        const int64_t r = (live ? row : row2) - p * R;
        const double kx = k_hat[3 * r], ky = k_hat[3 * r + 1], kz = k_hat[3 * r + 2];
        const double ex = e_hat[3 * r], ey = e_hat[3 * r + 1], ez = e_hat[3 * r + 2];
        const double sp = (w.tx * ex + w.ty * ey + w.tz * ez) >= 0.0 ? 1.0 : -1.0;
        const double tx = sp * w.tx, ty = sp * w.ty, tz = sp * w.tz;
        const bool is_slot = m < KNB && slot[m < KNB ? m : 0] >= 0;
        const bool is_own = m >= 16 && m < 23;
        const int jj = m < KNB ? m : 0;
        double dx = 0.0, dy = 0.0, dz = 0.0;
        if (is_slot) {
            dx = sg[jj][0];
            dy = sg[jj][1];
            dz = sg[jj][2];
        }
        double beta = 0.0, arg = 0.0;
        if (is_own) {
            beta = k * (kx * tx + ky * ty + kz * tz);
            arg = beta * (-0.5 * w.len + (m - 16 + 1) * D);
        } else if (is_slot) {
            arg = k * (kx * dx + ky * dy + kz * dz);
        }
        double sn, cs;
        sincos(arg, &sn, &cs);
        if (!live) continue;
        uint16_t* out = feat + (row - row0) * NF;
        if (is_slot) {
            const double vtx = sg[jj][4], vty = sg[jj][5], vtz = sg[jj][6];
            const double sv = (vtx * ex + vty * ey + vtz * ez) >= 0.0 ? 1.0 : -1.0;
            const double ux = sv * vtx, uy = sv * vty, uz = sv * vtz;
            const double ue = ux * ex + uy * ey + uz * ez;
            uint16_t* f = out + FOWN + FNB * jj;
            f[0] = fixed[jj][0];
            f[1] = d2bf((tx * dx + ty * dy + tz * dz) / d_c);
            f[2] = d2bf((ux * dx + uy * dy + uz * dz) / d_c);
            f[3] = d2bf(tx * ux + ty * uy + tz * uz);
            f[4] = d2bf(ue * cs);
            f[5] = d2bf(-ue * sn);
            f[6] = fixed[jj][1];
            f[7] = d2bf(kx * ux + ky * uy + kz * uz);
            f[8] = fixed[jj][2];
            f[9] = fixed[jj][3];
            f[10] = d2bf(1.0);
        } else if (m < KNB) {   // empty slot
            uint16_t* f = out + FOWN + FNB * m;
#pragma unroll
            for (int g = 0; g < FNB; ++g) f[g] = 0;
        } else if (is_own) {
            const double te = tx * ex + ty * ey + tz * ez;
            const double env = sinc_d(beta * D / 2.0);
            const double a = te * (env * env);
            const int q = m - 16;
            out[2 + 2 * q] = d2bf(a * cs);
            out[3 + 2 * q] = d2bf(-a * sn);
        } else if (m == 23) {
            out[0] = d2bf(10.0 * (w.len / lam - 0.5));
            out[1] = d2bf((double)cnt / 16.0);
        }
    }
}

// ------------------------------------------------------------------ currents <-> outputs
// Isolated response of wire w: b = Pinv_p u_p exp(+j k k_hat.c_p), raw rooftop
// order, FP64 accumulation over the stored inverse self block.
template <typename CZ>
__device__ __forceinline__ void isolated_response(const Wire& w, const CZ* __restrict__ P, const double* kh,
                                                  const double* eh, double k, c128 (&b)[7]) {
    const double te = w.tx * eh[0] + w.ty * eh[1] + w.tz * eh[2];
    const double beta = k * (kh[0] * w.tx + kh[1] * w.ty + kh[2] * w.tz);
    const double D = w.len / 8.0;
    const double sc = sinc_d(0.5 * beta * D);
    const double env = te * D * (sc * sc);
    c128 u[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        double sn, cs;
        sincos(beta * (-0.5 * w.len + (q + 1) * D), &sn, &cs);
        u[q] = c128{env * cs, -env * sn};
    }
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        c128 a{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 7; ++j) cfma(a, ccast<c128>(P[i * 7 + j]), u[j]);
        b[i] = a;
    }
}

template <typename CZ>
__global__ void k_targets(const Wire* __restrict__ wires, const int32_t* __restrict__ iperm, const CZ* __restrict__ Pinv,
                          int64_t n, int64_t R, const double* __restrict__ k_hat, const double* __restrict__ e_hat,
                          double k, const c128* __restrict__ X, float* __restrict__ Y) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n * R) return;
    const int64_t p = row / R, r = row - p * R;
    const int32_t ip = iperm[p];
    const Wire w = wires[ip];
    const double* kh = k_hat + 3 * r;
    const double* eh = e_hat + 3 * r;
    const bool flip = (w.tx * eh[0] + w.ty * eh[1] + w.tz * eh[2]) < 0.0;
    c128 b[7];
    isolated_response(w, Pinv + (int64_t)ip * 49, kh, eh, k, b);
    double sn, cs;
    sincos(k * (kh[0] * w.cx + kh[1] * w.cy + kh[2] * w.cz), &sn, &cs);
    const double sc = (flip ? -1.0 : 1.0) / X_SCALE;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const int qr = flip ? 6 - q : q;
        const c128 x = X[(p * 7 + qr) * R + r];
        const double dr = (x.re * cs - x.im * sn) - b[qr].re;
        const double di = (x.re * sn + x.im * cs) - b[qr].im;
        Y[row * NO + 2 * q] = (float)(sc * dr);
        Y[row * NO + 2 * q + 1] = (float)(sc * di);
    }
}

template <typename CZ>
__global__ void k_assemble(const Wire* __restrict__ wires, const int32_t* __restrict__ iperm,
                           const CZ* __restrict__ Pinv, int64_t R, int64_t row0, int64_t n_rows,
                           const double* __restrict__ k_hat, const double* __restrict__ e_hat, double k,
                           const float* __restrict__ Y, c128* __restrict__ X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows) return;
    const int64_t row = row0 + t;
    const int64_t p = row / R, r = row - p * R;
    const int32_t ip = iperm[p];
    const Wire w = wires[ip];
    const double* kh = k_hat + 3 * r;
    const double* eh = e_hat + 3 * r;
    const bool flip = (w.tx * eh[0] + w.ty * eh[1] + w.tz * eh[2]) < 0.0;
    c128 b[7];
    isolated_response(w, Pinv + (int64_t)ip * 49, kh, eh, k, b);
    double sn, cs;
    sincos(k * (kh[0] * w.cx + kh[1] * w.cy + kh[2] * w.cz), &sn, &cs);
    const double sc = (flip ? -1.0 : 1.0) * X_SCALE;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const int qr = flip ? 6 - q : q;
        const double dr = b[qr].re + sc * Y[t * NO + 2 * q];
        const double di = b[qr].im + sc * Y[t * NO + 2 * q + 1];
        // x = (b + d) exp(-j phase)
        X[(p * 7 + qr) * R + r] = c128{dr * cs + di * sn, di * cs - dr * sn};
    }
}

// ------------------------------------------------------------------ host side
// ------------------------------------------------------------------ learned neighbourhood inverse
// The same network as a block preconditioner: sample (wire i, slot s,
// column c) of a neighbourhood-inverse buffer predicts column c of the raw
// row block W_i[i, q] (q = N(i)[s]) in the canonical frames of i and q, from
// the neighbourhood's geometry alone; the predicted rows are symmetrised like
// the computed ones.  Canonical tangent tau = sigma t, sigma = +1 when the
// first nonzero of (t_z, t_y, t_x) is positive; S = sigma P maps rooftop
// coefficients to the canonical frame (P reverses the rooftops for sigma = -1).
// Rows: (i size + s) 7 + c, internal wire order i.
constexpr int NBF_HEAD = 24, NBF_MEM = 15;   // features: head, then 15 per neighbourhood member
constexpr double NBH_TARGET_SCALE = 0.05;    // targets: departures from the block-Jacobi blocks, times this

__device__ __forceinline__ double canon_sign(const Wire& w) {
    return (w.tz > 0.0 || (w.tz == 0.0 && (w.ty > 0.0 || (w.ty == 0.0 && w.tx > 0.0)))) ? 1.0 : -1.0;
}

// |d|/d_c, tau_x.d/d_c, tau_y.d/d_c, tau_x.tau_y, Re, Im exp(-j k |d|) with d = c_y - c_x
__device__ __forceinline__ void pair_feats(const Wire& x, double sx, const Wire& y, double sy, double k, double dc,
                                           double (&f)[6]) {
#pragma clang fp contract(off)
    const double dx = y.cx - x.cx, dy = y.cy - x.cy, dz = y.cz - x.cz;
    const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
    double s2 = xx + yy;
    s2 = s2 + zz;
    const double dist = sqrt(s2);
    const double xd = sx * ((x.tx * dx + x.ty * dy) + x.tz * dz);
    const double yd = sy * ((y.tx * dx + y.ty * dy) + y.tz * dz);
    const double tt = sx * sy * ((x.tx * y.tx + x.ty * y.ty) + x.tz * y.tz);
    const double ph = k * dist;
    f[0] = dist / dc;
    f[1] = xd / dc;
    f[2] = yd / dc;
    f[3] = tt;
    f[4] = cos(ph);
    f[5] = -sin(ph);
}

// One wave per (wire, slot): lanes 0..m-1 form the 15 features of one member
// each, lane 63 the head; the 192-entry row is staged in LDS and written for
// the 7 columns (one-hot c patched in) with coalesced stores.
__global__ __launch_bounds__(256) void k_nbhd_feat(const Wire* __restrict__ wires, const int32_t* __restrict__ nbt,
                                                   int size, int64_t n, int64_t row0, int64_t n_rows, double k,
                                                   double lam, double dc, uint16_t* __restrict__ feat) {
#pragma clang fp contract(off)
    __shared__ uint16_t fs[4][NF];
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t g = row0 / NB_W + (int64_t)blockIdx.x * 4 + w;   // rows 7 g .. 7 g + 6
    const int64_t i = g / size;
    const int s = (int)(g - i * size);
    if (i >= n || NB_W * g >= row0 + n_rows) return;   // wave-uniform
    for (int f = lane; f < NF; f += 64) fs[w][f] = 0;
    int32_t mem[8];
    int m = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        mem[t] = t < size ? nbt[i * size + t] : -1;
        m += mem[t] >= 0 ? 1 : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool live = s < m;
    if (live) {
        const Wire wp = wires[i];
        const int32_t q = mem[s];
        const Wire wq = wires[q];
        const double sp = canon_sign(wp), sq = canon_sign(wq);
        double f6[6];
        if (lane < m) {
            int32_t wt = mem[0];
#pragma unroll
            for (int t = 1; t < 8; ++t)
                if (t == lane) wt = mem[t];
            const Wire ww = wires[wt];
            const double sw = canon_sign(ww);
            uint16_t* o = &fs[w][NBF_HEAD + NBF_MEM * lane];
            o[0] = d2bf(1.0);
            o[1] = d2bf(10.0 * (ww.len / lam - 0.5));
            pair_feats(wp, sp, ww, sw, k, dc, f6);
#pragma unroll
            for (int j = 0; j < 6; ++j) o[2 + j] = d2bf(f6[j]);
            pair_feats(wq, sq, ww, sw, k, dc, f6);
#pragma unroll
            for (int j = 0; j < 6; ++j) o[8 + j] = d2bf(f6[j]);
            const double dx = ww.cx - wq.cx, dy = ww.cy - wq.cy, dz = ww.cz - wq.cz;
            const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
            double s2 = xx + yy;
            s2 = s2 + zz;
            o[14] = d2bf((wt == q || s2 <= dc * dc) ? 1.0 : 0.0);
        }
        if (lane == 63) {
            uint16_t* o = fs[w];
            o[7 + s] = d2bf(1.0);
            o[15] = d2bf(10.0 * (wp.len / lam - 0.5));
            o[16] = d2bf(10.0 * (wq.len / lam - 0.5));
            pair_feats(wp, sp, wq, sq, k, dc, f6);
#pragma unroll
            for (int j = 0; j < 6; ++j) o[17 + j] = d2bf(f6[j]);
            o[23] = d2bf(m / 8.0);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint16_t one = d2bf(1.0);
    for (int c = 0; c < NB_W; ++c) {
        const int64_t row = NB_W * g + c;
        if (row < row0 || row >= row0 + n_rows) continue;
        uint16_t* out = feat + (row - row0) * NF;
        for (int f = lane; f < NF; f += 64) out[f] = (live && f == c) ? one : fs[w][f];
    }
}

__device__ __forceinline__ int64_t block_pos(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                                             int64_t i, int32_t q) {
    int64_t p = -1;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
        if (col_idx[e] == q) p = e;
    return p;
}

// Targets of every row from a buffer of raw rows: y[2r], y[2r+1] = scale *
// (S_i (W - delta_iq Pinv_i) S_q)[r][c], the departure from the block-diagonal
// preconditioner (Pinv the inverse self blocks of the fill).
template <typename CZ>
__global__ void k_nbhd_targets(const Wire* __restrict__ wires, const int32_t* __restrict__ nbt, int size, int64_t n,
                               const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx,
                               const CZ* __restrict__ Mv, const CZ* __restrict__ Pinv, float* __restrict__ Y) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n * size * NB_W) return;
    const int64_t g = row / NB_W;
    const int c = (int)(row - g * NB_W);
    const int64_t i = g / size;
    const int s = (int)(g - i * size);
    float* y = Y + row * NO;
    const int32_t q = nbt[i * size + s];
    if (q < 0) {
#pragma unroll
        for (int r = 0; r < NO; ++r) y[r] = 0.f;
        return;
    }
    const int64_t pos = block_pos(row_ptr, col_idx, i, q);
    const double sp = canon_sign(wires[i]), sq = canon_sign(wires[q]);
    const int cq = sq > 0 ? c : NB_W - 1 - c;
    const double f = sp * sq * NBH_TARGET_SCALE;
#pragma unroll
    for (int r = 0; r < NB_W; ++r) {
        const int rp = sp > 0 ? r : NB_W - 1 - r;
        const CZ v = Mv[pos * NB_W * NB_W + rp * NB_W + cq];
        double re = (double)v.re, im = (double)v.im;
        if (q == i) {
            const CZ b = Pinv[i * NB_W * NB_W + rp * NB_W + cq];
            re -= (double)b.re;
            im -= (double)b.im;
        }
        y[2 * r] = (float)(f * re);
        y[2 * r + 1] = (float)(f * im);
    }
}

// Raw rows from network outputs (rows [row0, row0 + n_rows)): the inverse map of k_nbhd_targets.
template <typename CZ>
__global__ void k_nbhd_assemble(const Wire* __restrict__ wires, const int32_t* __restrict__ nbt, int size,
                                const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx, int64_t row0,
                                int64_t n_rows, const float* __restrict__ Y, const CZ* __restrict__ Pinv,
                                CZ* __restrict__ Mv) {
    using R = typename real_of<CZ>::type;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows) return;
    const int64_t row = row0 + t;
    const int64_t g = row / NB_W;
    const int c = (int)(row - g * NB_W);
    const int64_t i = g / size;
    const int s = (int)(g - i * size);
    const int32_t q = nbt[i * size + s];
    if (q < 0) return;
    const int64_t pos = block_pos(row_ptr, col_idx, i, q);
    const double sp = canon_sign(wires[i]), sq = canon_sign(wires[q]);
    const int cq = sq > 0 ? c : NB_W - 1 - c;
    const double f = sp * sq / NBH_TARGET_SCALE;
    const float* y = Y + t * NO;
#pragma unroll
    for (int r = 0; r < NB_W; ++r) {
        const int rp = sp > 0 ? r : NB_W - 1 - r;
        double re = f * (double)y[2 * r], im = f * (double)y[2 * r + 1];
        if (q == i) {
            const CZ b = Pinv[i * NB_W * NB_W + rp * NB_W + cq];
            re += (double)b.re;
            im += (double)b.im;
        }
        Mv[pos * NB_W * NB_W + rp * NB_W + cq] = CZ{(R)re, (R)im};
    }
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }
inline int64_t pad_rows(int64_t m, int64_t a) { return (m + a - 1) / a * a; }

struct TrainBufs {
    Packed pk;
    uint16_t *fT, *a1, *a2, *a3, *aT1, *aT2, *aT3, *dY, *dYT, *dZ3, *dZ2, *dZT3, *dZT2, *dZT1;
    float *z1, *z2, *z3, *part, *loss_part, *grad;
};

void carve_packed(Carve& cv, Packed& pk) {
    pk.wt1 = cv.take<uint16_t>(NH * NF);
    pk.wt2 = cv.take<uint16_t>(NH * NH);
    pk.wt3 = cv.take<uint16_t>(NH * NH);
    pk.wt4 = cv.take<uint16_t>(NOP * NH);
    pk.wn2 = cv.take<uint16_t>(NH * NH);
    pk.wn3 = cv.take<uint16_t>(NH * NH);
    pk.wn4 = cv.take<uint16_t>(NH * DYLD);
}

TrainBufs carve_train(Carve& cv, int64_t Mpad) {
    TrainBufs b{};
    carve_packed(cv, b.pk);
    b.fT = cv.take<uint16_t>(NF * Mpad);
    b.a1 = cv.take<uint16_t>(Mpad * NH);
    b.a2 = cv.take<uint16_t>(Mpad * NH);
    b.a3 = cv.take<uint16_t>(Mpad * NH);
    b.aT1 = cv.take<uint16_t>(NH * Mpad);
    b.aT2 = cv.take<uint16_t>(NH * Mpad);
    b.aT3 = cv.take<uint16_t>(NH * Mpad);
    b.z1 = cv.take<float>(Mpad * NH);
    b.z2 = cv.take<float>(Mpad * NH);
    b.z3 = cv.take<float>(Mpad * NH);
    b.dY = cv.take<uint16_t>(Mpad * DYLD);
    b.dYT = cv.take<uint16_t>(NOP * Mpad);
    b.dZ3 = cv.take<uint16_t>(Mpad * NH);
    b.dZ2 = cv.take<uint16_t>(Mpad * NH);
    b.dZT3 = cv.take<uint16_t>(NH * Mpad);
    b.dZT2 = cv.take<uint16_t>(NH * Mpad);
    b.dZT1 = cv.take<uint16_t>(NH * Mpad);
    b.part = cv.take<float>((size_t)(Mpad / SPLIT_ROWS) * NPARAM);
    b.loss_part = cv.take<float>(Mpad / 32);
    b.grad = cv.take<float>(NPARAM);
    return b;
}

struct FwdBufs {
    Packed pk;
    float* Y;
};

FwdBufs carve_fwd(Carve& cv, int64_t Mpad, bool with_y) {
    FwdBufs b{};
    carve_packed(cv, b.pk);
    b.Y = with_y ? cv.take<float>(Mpad * NO) : nullptr;
    return b;
}

chaff_status launch_pack(const float* theta, const Packed& pk, hipStream_t st) {
    hipLaunchKernelGGL(k_pack, dim3(nblk(NF * NH, 256), 7), dim3(256), 0, st, theta, pk);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

double layer_flops(int64_t m, int k, int n) { return 2.0 * (double)m * k * n; }

// Fused inference over rows [0, M): one persistent workgroup per CU.
chaff_status forward_fused(const float* theta, const Packed& pk, const uint16_t* feat, int64_t M, float* Y,
                           hipStream_t st) {
    static const bool attr = [] {
        return hipFuncSetAttribute((const void*)k_fwd_fused, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   FUSED_LDS) == hipSuccess;
    }();
    if (!attr) return fail(CHAFF_EHIP, "cannot reserve LDS for the fused forward kernel");
    const int64_t tiles = (M + 31) / 32;
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (tiles + 3) / 4));
    ProfScope ps("mlp_forward", st, layer_flops(M, NF, NH) + 2 * layer_flops(M, NH, NH) + layer_flops(M, NH, NO), true);
    hipLaunchKernelGGL(k_fwd_fused, dim3(grid), dim3(256), FUSED_LDS, st, feat, M, theta, pk, Y);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

}  // namespace

// ---------------------------------------------------------------- entry points (called from abi.cpp)

size_t mlp_workspace_bytes(int64_t rows, int32_t train) {
    Carve cv(nullptr, 0);
    if (train) carve_train(cv, pad_rows(rows, SPLIT_ROWS));
    else carve_fwd(cv, pad_rows(rows, ROWS_WG), false);
    return cv.off + 256;
}

chaff_status mlp_forward(const float* theta, const uint16_t* feat, int64_t M, float* Y, void* ws, size_t ws_bytes,
                         hipStream_t st) {
    Carve cv(ws, ws_bytes);
    FwdBufs b = carve_fwd(cv, pad_rows(M, ROWS_WG), false);
    if (!cv.ok()) return fail(CHAFF_EWORKSPACE, "mlp workspace too small");
    chaff_status s = launch_pack(theta, b.pk, st);
    if (s != CHAFF_OK) return s;
    return forward_fused(theta, b.pk, feat, M, Y, st);
}

chaff_status mlp_grad(const float* theta, const uint16_t* feat, const float* T, const int64_t* idx, int64_t M,
                      float* grad, float* loss, void* ws, size_t ws_bytes, hipStream_t st) {
    const int64_t Mpad = pad_rows(M, SPLIT_ROWS);
    Carve cv(ws, ws_bytes);
    TrainBufs b = carve_train(cv, Mpad);
    if (!cv.ok()) return fail(CHAFF_EWORKSPACE, "mlp workspace too small");
    if (!grad) grad = b.grad;
    chaff_status s = launch_pack(theta, b.pk, st);
    if (s != CHAFF_OK) return s;
    const unsigned grid = (unsigned)(Mpad / ROWS_WG);
    const int64_t nsplit = Mpad / SPLIT_ROWS;
    {
        ProfScope ps("mlp_grad", st, 3.0 * (layer_flops(M, NF, NH) + 2 * layer_flops(M, NH, NH) + layer_flops(M, NH, NO)),
                     true);
        hipLaunchKernelGGL(k_feat_t, dim3((unsigned)(Mpad / 64)), dim3(256), 0, st, feat, idx, M, Mpad, b.fT);
        FwdArgs a{};
        a.M = M;
        a.Mpad = Mpad;
        a.a_idx = idx;
        a.A = feat; a.lda = NF; a.Wt = b.pk.wt1; a.K = NF; a.bias = theta + OB1;
        a.a_out = b.a1; a.z_out = b.z1; a.aT_out = b.aT1;
        hipLaunchKernelGGL((k_fwd<false, true>), dim3(grid), dim3(256), 0, st, a);
        a.a_idx = nullptr;
        a.A = b.a1; a.lda = NH; a.Wt = b.pk.wt2; a.K = NH; a.bias = theta + OB2;
        a.a_out = b.a2; a.z_out = b.z2; a.aT_out = b.aT2;
        hipLaunchKernelGGL((k_fwd<false, true>), dim3(grid), dim3(256), 0, st, a);
        a.A = b.a2; a.Wt = b.pk.wt3; a.bias = theta + OB3;
        a.a_out = b.a3; a.z_out = b.z3; a.aT_out = b.aT3;
        hipLaunchKernelGGL((k_fwd<false, true>), dim3(grid), dim3(256), 0, st, a);
        a.A = b.a3; a.Wt = b.pk.wt4; a.bias = theta + OB4; a.a_out = nullptr; a.z_out = nullptr; a.aT_out = nullptr;
        a.t_idx = idx; a.T = T; a.dY = b.dY; a.dYT = b.dYT; a.loss_part = b.loss_part;
        hipLaunchKernelGGL((k_fwd<true, true>), dim3(grid), dim3(256), 0, st, a);

        BwdArgs d{};
        d.Mpad = Mpad;
        d.dZ = b.dY; d.lda = DYLD; d.K = DYLD; d.Wn = b.pk.wn4; d.z_prev = b.z3; d.dZ_out = b.dZ3; d.dZT_out = b.dZT3;
        hipLaunchKernelGGL(k_bwd, dim3(grid), dim3(256), 0, st, d);
        d.dZ = b.dZ3; d.lda = NH; d.K = NH; d.Wn = b.pk.wn3; d.z_prev = b.z2; d.dZ_out = b.dZ2; d.dZT_out = b.dZT2;
        hipLaunchKernelGGL(k_bwd, dim3(grid), dim3(256), 0, st, d);
        d.dZ = b.dZ2; d.Wn = b.pk.wn2; d.z_prev = b.z1; d.dZ_out = nullptr; d.dZT_out = b.dZT1;
        hipLaunchKernelGGL(k_bwd, dim3(grid), dim3(256), 0, st, d);

        const unsigned ns = (unsigned)nsplit;
        hipLaunchKernelGGL((k_wgrad<4>), dim3(NF / 16, NH / 64, ns), dim3(64), 0, st, (const uint16_t*)b.fT,
                           (const uint16_t*)b.dZT1, Mpad, NH, OW1, b.part);
        hipLaunchKernelGGL((k_wgrad<4>), dim3(NH / 16, NH / 64, ns), dim3(64), 0, st, (const uint16_t*)b.aT1,
                           (const uint16_t*)b.dZT2, Mpad, NH, OW2, b.part);
        hipLaunchKernelGGL((k_wgrad<4>), dim3(NH / 16, NH / 64, ns), dim3(64), 0, st, (const uint16_t*)b.aT2,
                           (const uint16_t*)b.dZT3, Mpad, NH, OW3, b.part);
        hipLaunchKernelGGL((k_wgrad<1>), dim3(NH / 16, 1, ns), dim3(64), 0, st, (const uint16_t*)b.aT3,
                           (const uint16_t*)b.dYT, Mpad, NO, OW4, b.part);
        hipLaunchKernelGGL(k_bgrad, dim3(NO + 3 * NH, ns), dim3(64), 0, st, (const uint16_t*)b.dYT,
                           (const uint16_t*)b.dZT3, (const uint16_t*)b.dZT2, (const uint16_t*)b.dZT1, Mpad, b.part);
        const float scale = (float)(1.0 / ((double)M * NO));
        hipLaunchKernelGGL(k_reduce, dim3(nblk(NPARAM, 256) + 1), dim3(256), 0, st, (const float*)b.part, nsplit,
                           scale, grad, (const float*)b.loss_part, Mpad / 32, loss);
    }
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t t, float lr, float b1, float b2,
                      float eps, hipStream_t st) {
    const double bc1 = 1.0 - std::pow((double)b1, (double)t), bc2 = 1.0 - std::pow((double)b2, (double)t);
    ProfScope ps("mlp_adam", st, 4.0 * 7 * NPARAM);
    hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAM, 256)), dim3(256), 0, st, theta, m, v, grad, lr, b1, b2, eps,
                       (float)bc1, (float)bc2);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status mlp_train_step(float* theta, float* m, float* v, int32_t t, float lr, float b1, float b2, float eps,
                            const uint16_t* feat, const float* T, const int64_t* idx, int64_t M, float* loss, void* ws,
                            size_t ws_bytes, hipStream_t st) {
    const int64_t Mpad = pad_rows(M, SPLIT_ROWS);
    Carve cv(ws, ws_bytes);
    TrainBufs b = carve_train(cv, Mpad);
    if (!cv.ok()) return fail(CHAFF_EWORKSPACE, "mlp workspace too small");
    chaff_status s = mlp_grad(theta, feat, T, idx, M, b.grad, loss, ws, ws_bytes, st);
    if (s != CHAFF_OK) return s;
    return mlp_adam(theta, m, v, b.grad, t, lr, b1, b2, eps, st);
}

chaff_status mlp_features(Cloud* c, const double* k_hat, const double* e_hat, int64_t R, int64_t row0, int64_t n_rows,
                          uint16_t* feat, hipStream_t st) {
    if (n_rows == 0) return CHAFF_OK;
    const double k = 2.0 * 3.14159265358979323846 / c->wavelength;
    ProfScope ps("mlp_features", st, (double)n_rows * NF * 2.0);
    const int64_t n_wires = (row0 + n_rows - 1) / R - row0 / R + 1;
    hipLaunchKernelGGL(k_features, dim3((unsigned)n_wires), dim3(64), 0, st, (const Wire*)c->wires,
                       (const int32_t*)c->perm, (const int32_t*)c->iperm, (const int64_t*)c->row_ptr,
                       (const int32_t*)c->col_idx, R, row0, n_rows, k_hat, e_hat, k, c->wavelength, c->d_c, feat);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status mlp_targets(Cloud* c, chaff_prec prec, const void* Pinv, const double* k_hat, const double* e_hat,
                         int64_t R, const void* X, float* Y, hipStream_t st) {
    const double k = 2.0 * 3.14159265358979323846 / c->wavelength;
    ProfScope ps("mlp_targets", st, (double)c->n * R * (7 * 16 + NO * 4));
    if (prec == CHAFF_C64)
        hipLaunchKernelGGL(k_targets<c64>, dim3(nblk(c->n * R, 256)), dim3(256), 0, st, (const Wire*)c->wires,
                           (const int32_t*)c->iperm, (const c64*)Pinv, c->n, R, k_hat, e_hat, k, (const c128*)X, Y);
    else
        hipLaunchKernelGGL(k_targets<c128>, dim3(nblk(c->n * R, 256)), dim3(256), 0, st, (const Wire*)c->wires,
                           (const int32_t*)c->iperm, (const c128*)Pinv, c->n, R, k_hat, e_hat, k, (const c128*)X, Y);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

constexpr int64_t GUESS_CHUNK = 1 << 18;  // rows per features/forward pass

size_t mlp_guess_workspace_bytes(const Cloud* c, int64_t R) {
    const int64_t rows = std::min<int64_t>(c->n * R, GUESS_CHUNK);
    Carve cv(nullptr, 0);
    carve_fwd(cv, pad_rows(rows, ROWS_WG), true);
    cv.take<uint16_t>((size_t)pad_rows(rows, ROWS_WG) * NF);
    return cv.off + 256;
}

chaff_status mlp_guess(Cloud* c, chaff_prec prec, const void* Pinv, const float* theta, const double* k_hat,
                       const double* e_hat, int64_t R, void* X, void* ws, size_t ws_bytes, hipStream_t st) {
    const int64_t total = c->n * R;
    const int64_t chunk = std::min<int64_t>(total, GUESS_CHUNK);
    Carve cv(ws, ws_bytes);
    FwdBufs b = carve_fwd(cv, pad_rows(chunk, ROWS_WG), true);
    uint16_t* feat = cv.take<uint16_t>((size_t)pad_rows(chunk, ROWS_WG) * NF);
    if (!cv.ok()) return fail(CHAFF_EWORKSPACE, "mlp guess workspace too small");
    chaff_status s = launch_pack(theta, b.pk, st);
    if (s != CHAFF_OK) return s;
    const double k = 2.0 * 3.14159265358979323846 / c->wavelength;
    for (int64_t r0 = 0; r0 < total; r0 += chunk) {
        const int64_t nr = std::min(chunk, total - r0);
        s = mlp_features(c, k_hat, e_hat, R, r0, nr, feat, st);
        if (s != CHAFF_OK) return s;
        s = forward_fused(theta, b.pk, feat, nr, b.Y, st);
        if (s != CHAFF_OK) return s;
        ProfScope ps("mlp_assemble", st, (double)nr * (NO * 4 + 7 * 16) + (double)nr / R * 49 * (prec == CHAFF_C64 ? 8 : 16));
        if (prec == CHAFF_C64)
            hipLaunchKernelGGL(k_assemble<c64>, dim3(nblk(nr, 256)), dim3(256), 0, st, (const Wire*)c->wires,
                               (const int32_t*)c->iperm, (const c64*)Pinv, R, r0, nr, k_hat, e_hat, k,
                               (const float*)b.Y, (c128*)X);
        else
            hipLaunchKernelGGL(k_assemble<c128>, dim3(nblk(nr, 256)), dim3(256), 0, st, (const Wire*)c->wires,
                               (const int32_t*)c->iperm, (const c128*)Pinv, R, r0, nr, k_hat, e_hat, k,
                               (const float*)b.Y, (c128*)X);
        CHAFF_LAUNCH_CHECK();
    }
    return CHAFF_OK;
}

// ---------------------------------------------------------------- learned neighbourhood inverse (host)

constexpr int64_t NBH_MLP_CHUNK = 7 * (1 << 15);   // rows per features/forward pass (whole wire slots)

chaff_status nbhd_mlp_features_n(Cloud* c, int size, const void* M, int64_t row0, int64_t n_rows, uint16_t* feat,
                                 hipStream_t st) {
    if (n_rows == 0 || c->n == 0) return CHAFF_OK;
    const int32_t* nbt = reinterpret_cast<const int32_t*>(static_cast<const char*>(M) + NBH_HEADER);
    const double k = 2.0 * 3.14159265358979323846 / c->wavelength;
    const int64_t g0 = row0 / NB_W, g1 = (row0 + n_rows - 1) / NB_W;
    ProfScope ps("nbhd_mlp_features", st, (double)n_rows * NF * 2.0);
    hipLaunchKernelGGL(k_nbhd_feat, dim3(nblk(g1 - g0 + 1, 4)), dim3(256), 0, st, (const Wire*)c->wires, nbt, size,
                       c->n, row0, n_rows, k, c->wavelength, c->d_c, feat);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status nbhd_mlp_features(Cloud* c, const void* M, int64_t row0, int64_t n_rows, uint16_t* feat, hipStream_t st) {
    NbhdHeader h{};
    chaff_status s = nbhd_header(c, M, &h, st);
    if (s != CHAFF_OK) return s;
    if (row0 + n_rows > c->n * h.size * NB_W)
        return fail(CHAFF_EINVAL, "rows beyond the buffer's N * size * 7 samples");
    return nbhd_mlp_features_n(c, h.size, M, row0, n_rows, feat, st);
}

chaff_status nbhd_mlp_targets(Cloud* c, chaff_prec prec, const void* M, const void* Pinv, float* Y, hipStream_t st) {
    NbhdHeader h{};
    chaff_status s = nbhd_header(c, M, &h, st);
    if (s != CHAFF_OK) return s;
    if (!h.raw || h.prec != (int32_t)prec)
        return fail(CHAFF_EINVAL, "targets need a buffer of raw rows (chaff_nbhd_raw_rows) of the same precision");
    const int64_t rows = c->n * h.size * NB_W;
    if (rows == 0) return CHAFF_OK;
    const int32_t* nbt = reinterpret_cast<const int32_t*>(static_cast<const char*>(M) + NBH_HEADER);
    const char* vals = static_cast<const char*>(M) + nbhd_blocks_offset(c->n, h.size);
    if (prec == CHAFF_C64)
        hipLaunchKernelGGL(k_nbhd_targets<c64>, dim3(nblk(rows, 256)), dim3(256), 0, st, (const Wire*)c->wires, nbt,
                           h.size, c->n, (const int64_t*)c->row_ptr, (const int32_t*)c->col_idx, (const c64*)vals,
                           (const c64*)Pinv, Y);
    else
        hipLaunchKernelGGL(k_nbhd_targets<c128>, dim3(nblk(rows, 256)), dim3(256), 0, st, (const Wire*)c->wires, nbt,
                           h.size, c->n, (const int64_t*)c->row_ptr, (const int32_t*)c->col_idx, (const c128*)vals,
                           (const c128*)Pinv, Y);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

size_t nbhd_mlp_workspace_bytes(const Cloud* c, int size) {
    const int64_t rows = std::max<int64_t>(1, std::min<int64_t>(c->n * size * NB_W, NBH_MLP_CHUNK));
    Carve cv(nullptr, 0);
    carve_fwd(cv, pad_rows(rows, ROWS_WG), true);
    cv.take<uint16_t>((size_t)pad_rows(rows, ROWS_WG) * NF);
    return cv.off + 256;
}

chaff_status nbhd_mlp_precond(Cloud* c, chaff_prec prec, int size, const float* theta, const void* Pinv, void* M,
                              void* ws, size_t ws_bytes, hipStream_t st) {
    chaff_status s = nbhd_begin(c, prec, size, false, M, st);
    if (s != CHAFF_OK || c->n == 0) return s;
    const int64_t total = c->n * size * NB_W;
    const int64_t chunk = std::min<int64_t>(total, NBH_MLP_CHUNK);
    Carve cv(ws, ws_bytes);
    FwdBufs b = carve_fwd(cv, pad_rows(chunk, ROWS_WG), true);
    uint16_t* feat = cv.take<uint16_t>((size_t)pad_rows(chunk, ROWS_WG) * NF);
    if (!cv.ok()) return fail(CHAFF_EWORKSPACE, "learned preconditioner workspace too small");
    s = launch_pack(theta, b.pk, st);
    if (s != CHAFF_OK) return s;
    const int32_t* nbt = reinterpret_cast<const int32_t*>(static_cast<const char*>(M) + NBH_HEADER);
    char* vals = static_cast<char*>(M) + nbhd_blocks_offset(c->n, size);
    for (int64_t r0 = 0; r0 < total; r0 += chunk) {
        const int64_t nr = std::min(chunk, total - r0);
        s = nbhd_mlp_features_n(c, size, M, r0, nr, feat, st);
        if (s != CHAFF_OK) return s;
        s = forward_fused(theta, b.pk, feat, nr, b.Y, st);
        if (s != CHAFF_OK) return s;
        ProfScope ps("nbhd_mlp_assemble", st, (double)nr * (NO * 4 + 7 * (prec == CHAFF_C64 ? 8 : 16)));
        if (prec == CHAFF_C64)
            hipLaunchKernelGGL(k_nbhd_assemble<c64>, dim3(nblk(nr, 256)), dim3(256), 0, st, (const Wire*)c->wires, nbt,
                               size, (const int64_t*)c->row_ptr, (const int32_t*)c->col_idx, r0, nr,
                               (const float*)b.Y, (const c64*)Pinv, (c64*)vals);
        else
            hipLaunchKernelGGL(k_nbhd_assemble<c128>, dim3(nblk(nr, 256)), dim3(256), 0, st, (const Wire*)c->wires,
                               nbt, size, (const int64_t*)c->row_ptr, (const int32_t*)c->col_idx, r0, nr,
                               (const float*)b.Y, (const c128*)Pinv, (c128*)vals);
        CHAFF_LAUNCH_CHECK();
    }
    s = nbhd_symmetrise(c, prec, vals, st);
    if (s != CHAFF_OK) return s;
    CHAFF_HIP(hipStreamSynchronize(st));
    return CHAFF_OK;
}

}  // namespace chaff
