// Block-sparse products and the multi-RHS Krylov solvers with FP64
// iterative refinement (Sec. II-B: iterative solve of the S-NFC system with a
// block-diagonal preconditioner; matvec cost O(b_mean N)).
//
// Included by krylov7.hip and krylov19.hip, once per rooftop count per wire:
// CHAFF_KNB unknowns per wire (7 for 8 segments, 19 for the 20 segments of
// the paper's own discretisation), inside namespace chaff::CHAFF_KNS.  The
// matrix-core forms of the product and the cluster preconditioner exist for
// 7 unknowns per wire only.
//
// Layout: every vector block is row-major [N*NB][s] in the internal (Morton)
// wire order, so the NB x s slab of one wire is contiguous and a column tile
// of s right-hand sides is read with unit stride.  Systems are independent
// per (cloud, RHS); all of them advance in lockstep so that each sparse
// product reads Z once for every right-hand side, while dot products are
// reduced per cloud over fixed row chunks in a fixed order (deterministic).
#include "common.hpp"
#include "precond.hpp"
#include "prof.hpp"
#include "tune.hpp"

#include <algorithm>
#include <chrono>
#include <mutex>
#include <type_traits>
#include <cstdio>
#include <cstdlib>

#ifndef CHAFF_KNB
#error "define CHAFF_KNB (unknowns per wire) and CHAFF_KNS (namespace) before including krylov_impl.hpp"
#endif

namespace chaff {
namespace CHAFF_KNS {

constexpr int NB = CHAFF_KNB;         // rooftop unknowns per wire
constexpr int NSEG = NB + 1;          // segments per wire
constexpr int NB2 = NB * NB;          // complex entries per block

constexpr double PI_K = 3.14159265358979323846;
constexpr int NXCD = 8;   // XCDs per MI355X; workgroup ids are dealt to them round-robin

// ------------------------------------------------------------------ SpMM
// MODE 0: Y = Z X    MODE 1: Y = B - Z X    MODE 2: Y += Z X
// DIAG: the pattern is the block diagonal (block i of Z applied to wire i).

template <typename CY> struct acc_t { using R = typename real_of<CY>::type; };

// Variant 0: lanes -> (block row, output row q); one RHS column per grid.y.
template <typename CZ, typename CX, typename CY, int MODE, bool DIAG>
__global__ __launch_bounds__(256) void k_spmm_rowq(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx,
                                                   const CZ* __restrict__ Z, const CX* __restrict__ X,
                                                   const CY* __restrict__ B, CY* __restrict__ Y,
                                                   int64_t n, int64_t s) {
    using R = typename real_of<CY>::type;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / NB;
    const int q = (int)(t - i * NB);
    const int64_t r = blockIdx.y;
    if (i >= n) return;
    const int64_t e0 = DIAG ? i : row_ptr[i];
    const int64_t e1 = DIAG ? i + 1 : row_ptr[i + 1];
    cplx<R> acc = {0, 0};
    // the column index and Z row of the next block are requested one block ahead
    int64_t col_n = DIAG ? i : (e0 < e1 ? col_idx[e0] : 0);
    CZ zn[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) zn[k] = e0 < e1 ? Z[e0 * NB2 + q * NB + k] : CZ{0, 0};
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t col = col_n;
        CZ zc[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) zc[k] = zn[k];
        if (e + 1 < e1) {
            if (!DIAG) col_n = col_idx[e + 1];
#pragma unroll
            for (int k = 0; k < NB; ++k) zn[k] = Z[(e + 1) * NB2 + q * NB + k];
        }
        const CX* xb = X + col * NB * s + r;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            cplx<R> z = ccast<cplx<R>>(zc[k]);
            cplx<R> x = ccast<cplx<R>>(xb[k * s]);
            cfma(acc, z, x);
        }
    }
    const int64_t o = (i * NB + q) * s + r;
    if (MODE == 0) Y[o] = ccast<CY>(acc);
    if (MODE == 1) Y[o] = ccast<CY>(csub(ccast<cplx<R>>(B[o]), acc));
    if (MODE == 2) Y[o] = ccast<CY>(cadd(ccast<cplx<R>>(Y[o]), acc));
}

// Variant 5: seven lanes per block row (lane = output row q), each lane
// accumulating SC RHS columns.  Every row of Z is loaded by exactly one lane
// once per product (the tile variants load each block once per column lane),
// and the seven lanes of a block row share the gathered X slab through L1.
// For small RHS counts the product then streams Z once, at full width.
template <typename CZ, typename CX, typename CY, int MODE, int SC, bool VEC>
__global__ __launch_bounds__(256) void k_spmm_rowq_multi(const int64_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col_idx,
                                                         const CZ* __restrict__ Z, const CX* __restrict__ X,
                                                         const CY* __restrict__ B, CY* __restrict__ Y,
                                                         int64_t n, int64_t s) {
    using R = typename real_of<CY>::type;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / NB;
    const int q = (int)(t - i * NB);
    const int64_t r0 = (int64_t)blockIdx.y * SC;
    if (i >= n) return;
    const int nc = (int)(s - r0 < SC ? s - r0 : SC);
    cplx<R> acc[SC];
#pragma unroll
    for (int c = 0; c < SC; ++c) acc[c] = {0, 0};
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    // the column index and Z row of the next block are requested one block ahead
    int64_t col_n = e0 < e1 ? col_idx[e0] : 0;
    CZ zn[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) zn[k] = e0 < e1 ? Z[e0 * NB2 + q * NB + k] : CZ{0, 0};
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t col = col_n;
        cplx<R> z[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) z[k] = ccast<cplx<R>>(zn[k]);
        if (e + 1 < e1) {
            col_n = col_idx[e + 1];
#pragma unroll
            for (int k = 0; k < NB; ++k) zn[k] = Z[(e + 1) * NB2 + q * NB + k];
        }
        const CX* xb = X + col * NB * s + r0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            bool done = false;
            if constexpr (VEC && SC >= 2) {   // pairs of columns in one 16-byte load (s and r0 even)
                if (nc == SC) {
                    const float4* xv = reinterpret_cast<const float4*>(xb + k * s);
#pragma unroll
                    for (int c = 0; c < SC; c += 2) {
                        const float4 v = xv[c / 2];
                        cfma(acc[c], z[k], cplx<R>{(R)v.x, (R)v.y});
                        cfma(acc[c + 1], z[k], cplx<R>{(R)v.z, (R)v.w});
                    }
                    done = true;
                }
            }
            if (done) {
            } else if (nc == SC) {
#pragma unroll
                for (int c = 0; c < SC; ++c) cfma(acc[c], z[k], ccast<cplx<R>>(xb[k * s + c]));
            } else {
#pragma unroll
                for (int c = 0; c < SC; ++c)
                    if (c < nc) cfma(acc[c], z[k], ccast<cplx<R>>(xb[k * s + c]));
            }
        }
    }
    const int64_t o = (i * NB + q) * s + r0;
#pragma unroll
    for (int c = 0; c < SC; ++c) {
        if (c >= nc) break;
        if (MODE == 0) Y[o + c] = ccast<CY>(acc[c]);
        if (MODE == 1) Y[o + c] = ccast<CY>(csub(ccast<cplx<R>>(B[o + c]), acc[c]));
        if (MODE == 2) Y[o + c] = ccast<CY>(cadd(ccast<cplx<R>>(Y[o + c]), acc[c]));
    }
}

// Variant 6: one wave per NR block rows and RHS tile of S columns.  The wave
// stages each 7x7 block in LDS with one coalesced load (prefetched one block
// ahead so the HBM latency overlaps the arithmetic of the previous block),
// lane (row sub, group g, column c) applies the block columns k = g, g + G,
// ... (G = 64/(NR S)) to its RHS column, and the G partial sums of a column
// are combined with cross-lane adds.  Z is read once per product.
// With XCD set, consecutive workgroup ids (dealt round-robin to the eight XCDs)
// are mapped so that XCD x walks the contiguous Morton range of row groups
// [x G/8, (x+1) G/8): the neighbour slabs a row gathers then stay in that
// XCD's L2.
template <typename CZ, typename CX, typename CY, int MODE, int S, int NR, bool XCD>
__global__ __launch_bounds__(64) void k_spmm_wave_row(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col_idx,
                                                      const CZ* __restrict__ Z, const CX* __restrict__ X,
                                                      const CY* __restrict__ B, CY* __restrict__ Y,
                                                      int64_t n, int64_t s) {
    using R = typename real_of<CY>::type;
    using ZT = cplx<R>;   // blocks are staged in the accumulation type: converted once per entry
    constexpr int G = 64 / (S * NR);
    constexpr int KK = (NB + G - 1) / G;
    __shared__ ZT zs[2][NR][NB2];
    const int lane = threadIdx.x;
    const int sub = lane / (S * G), g = (lane / S) % G, c = lane % S;
    int64_t grp = blockIdx.x;
    if (XCD) {
        const int64_t n_grp = (n + NR - 1) / NR;
        const int64_t per_xcd = (n_grp + NXCD - 1) / NXCD;
        grp = (int64_t)(blockIdx.x % NXCD) * per_xcd + blockIdx.x / NXCD;
        if (grp >= n_grp) return;   // uniform over the (single-wave) workgroup
    }
    const int64_t i = grp * NR + sub;
    const int64_t r = (int64_t)blockIdx.y * S + c;
    const bool live = r < s && i < n;
    const int64_t rc = r < s ? r : 0;
    // per row sub: edge range (wave-uniform loop over the longest row)
    int64_t eb[NR], ee[NR];
    int64_t len = 0;
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int64_t iu = grp * NR + u;
        eb[u] = iu < n ? row_ptr[iu] : 0;
        ee[u] = iu < n ? row_ptr[iu + 1] : 0;
        len = ee[u] - eb[u] > len ? ee[u] - eb[u] : len;
    }
    cplx<R> acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = {0, 0};
    // lane l < 49 loads entry l of the current block of every row sub
    CZ zn[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) zn[u] = (lane < NB2 && len > 0 && eb[u] < ee[u]) ? Z[eb[u] * NB2 + lane] : CZ{0, 0};
    for (int64_t t = 0; t < len; ++t) {
        const int buf = (int)(t & 1);
        if (lane < NB2) {
#pragma unroll
            for (int u = 0; u < NR; ++u) zs[buf][u][lane] = ccast<ZT>(zn[u]);
        }
        if (t + 1 < len && lane < NB2) {
#pragma unroll
            for (int u = 0; u < NR; ++u)
                if (eb[u] + t + 1 < ee[u]) zn[u] = Z[(eb[u] + t + 1) * NB2 + lane];
        }
        const int64_t e = eb[sub] + t;
        const bool have = e < ee[sub];
        cplx<R> x[KK];
        if (have) {
            const CX* xb = X + (int64_t)col_idx[e] * NB * s + rc;
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const int k = g + kk * G;
                x[kk] = k < NB ? ccast<cplx<R>>(xb[k * s]) : cplx<R>{0, 0};
            }
        }
        __syncthreads();
        if (have) {
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const int k = g + kk * G;
                if (k < NB) {
#pragma unroll
                    for (int q = 0; q < NB; ++q) cfma(acc[q], zs[buf][sub][q * NB + k], x[kk]);
                }
            }
        }
    }
#pragma unroll
    for (int off = S; off < S * G; off <<= 1)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            acc[q].re += __shfl_xor(acc[q].re, off, 64);
            acc[q].im += __shfl_xor(acc[q].im, off, 64);
        }
    if (g == 0 && live) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int64_t o = (i * NB + q) * s + r;
            if (MODE == 0) Y[o] = ccast<CY>(acc[q]);
            if (MODE == 1) Y[o] = ccast<CY>(csub(ccast<cplx<R>>(B[o]), acc[q]));
            if (MODE == 2) Y[o] = ccast<CY>(cadd(ccast<cplx<R>>(Y[o]), acc[q]));
        }
    }
}

// Variant 1: lanes -> (block row sub-index, RHS column); ST columns per row,
// each thread produces the 7 outputs of its (row, column).
template <typename CZ, typename CX, typename CY, int MODE, bool DIAG, int ST>
__global__ __launch_bounds__(256) void k_spmm_tile(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx,
                                                   const CZ* __restrict__ Z, const CX* __restrict__ X,
                                                   const CY* __restrict__ B, CY* __restrict__ Y,
                                                   int64_t n, int64_t s) {
    using R = typename real_of<CY>::type;
    const int rows_per_block = 256 / ST;
    const int64_t i = (int64_t)blockIdx.x * rows_per_block + threadIdx.x / ST;
    const int64_t r = (int64_t)blockIdx.y * ST + (threadIdx.x % ST);
    if (i >= n || r >= s) return;
    const int64_t e0 = DIAG ? i : row_ptr[i];
    const int64_t e1 = DIAG ? i + 1 : row_ptr[i + 1];
    cplx<R> acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = {0, 0};
    for (int64_t e = e0; e < e1; ++e) {
        const int64_t col = DIAG ? i : col_idx[e];
        const CZ* zb = Z + e * NB2;
        const CX* xb = X + col * NB * s + r;
        cplx<R> x[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) x[k] = ccast<cplx<R>>(xb[k * s]);
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int k = 0; k < NB; ++k) cfma(acc[q], ccast<cplx<R>>(zb[q * NB + k]), x[k]);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int64_t o = (i * NB + q) * s + r;
        if (MODE == 0) Y[o] = ccast<CY>(acc[q]);
        if (MODE == 1) Y[o] = ccast<CY>(csub(ccast<cplx<R>>(B[o]), acc[q]));
        if (MODE == 2) Y[o] = ccast<CY>(cadd(ccast<cplx<R>>(Y[o]), acc[q]));
    }
}

// Variant 3/4: the tile kernel with an XCD-aware workgroup order.  Workgroups
// are dispatched round-robin over the 8 XCDs (id % 8), each with its own L2;
// remapping id -> (row tile, column tile) so that XCD x walks rows
// [x*n/8, (x+1)*n/8) in Morton order keeps the neighbour slabs a row gathers
// inside that XCD's L2 while its neighbours are being processed.
template <typename CZ, typename CX, typename CY, int MODE, int ST>
__global__ __launch_bounds__(256) void k_spmm_xcd(const int64_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col_idx,
                                                  const CZ* __restrict__ Z, const CX* __restrict__ X,
                                                  const CY* __restrict__ B, CY* __restrict__ Y,
                                                  int64_t n, int64_t s, int64_t row_tiles, int col_tiles) {
    using R = typename real_of<CY>::type;
    const int rows_per_block = 256 / ST;
    const int64_t id = blockIdx.x;
    const int xcd = (int)(id % NXCD);
    const int64_t local = id / NXCD;
    const int64_t per_xcd = (row_tiles + NXCD - 1) / NXCD;
    const int64_t tile = (int64_t)xcd * per_xcd + local / col_tiles;
    const int ctile = (int)(local % col_tiles);
    if (tile >= row_tiles) return;
    const int sub = ST == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / ST);
    const int64_t i = tile * rows_per_block + sub;
    const int64_t r = (int64_t)ctile * ST + (threadIdx.x % ST);
    if (i >= n) return;
    const bool live = r < s;
    const int64_t rc = live ? r : 0;
    cplx<R> acc[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[q] = {0, 0};
    const int64_t e1 = row_ptr[i + 1];
    for (int64_t e = row_ptr[i]; e < e1; ++e) {
        const int64_t col = col_idx[e];
        const CZ* zb = Z + e * NB2;
        const CX* xb = X + col * NB * s + rc;
        cplx<R> x[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) x[k] = ccast<cplx<R>>(xb[k * s]);
#pragma unroll
        for (int q = 0; q < NB; ++q)
#pragma unroll
            for (int k = 0; k < NB; ++k) cfma(acc[q], ccast<cplx<R>>(zb[q * NB + k]), x[k]);
    }
    if (!live) return;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int64_t o = (i * NB + q) * s + r;
        if (MODE == 0) Y[o] = ccast<CY>(acc[q]);
        if (MODE == 1) Y[o] = ccast<CY>(csub(ccast<cplx<R>>(B[o]), acc[q]));
        if (MODE == 2) Y[o] = ccast<CY>(cadd(ccast<cplx<R>>(Y[o]), acc[q]));
    }
}

// default when nothing was tuned: one row per lane for a single RHS, else the
// XCD-aware tile order
static int default_variant(int64_t s) { return s == 1 ? 0 : 3; }

static int spmm_tile_width(int64_t s) {
    int st = 1;
    while (st < s && st < 64) st <<= 1;
    return st;
}
// RHS columns per wave of the COCG product (at least 8: at most 8 groups of block columns)
static int cocg_width(int64_t s) { return spmm_tile_width(s) < 8 ? 8 : spmm_tile_width(s); }

// variant: 0 = rowq, 1 = tile (ST from s), 2 = tile with ST halved (more rows per wave),
// 3 = tile in XCD-aware order, 4 = XCD-aware with ST halved, 5 = rowq with up to 16
// columns per lane, 6 = one wave per block row with the block staged in LDS, 7 = 6 in
// XCD-aware order
template <typename CZ, typename CX, typename CY, int MODE, bool DIAG>
static chaff_status spmm_launch(const int64_t* row_ptr, const int32_t* col_idx, const CZ* Z, const CX* X,
                                const CY* B, CY* Y, int64_t n, int64_t nnzb, int64_t s, int variant,
                                hipStream_t st, const char* tag = "spmm") {
    if (n == 0 || s == 0) return CHAFF_OK;
    // algorithmic HBM bytes: Z (and its indices) once, X once, Y once (+ B or Y read for MODE 1/2)
    const double zb = DIAG ? (double)sizeof(CZ) * NB2 * n
                           : ((double)sizeof(CZ) * NB2 + 4.0) * (double)nnzb + 8.0 * (n + 1);
    const double vb = 7.0 * n * s * ((double)sizeof(CX) + sizeof(CY) + (MODE == 0 ? 0.0 : (double)sizeof(CY)));
    ProfScope ps(tag, st, zb + vb, false);
    if (variant < 0) {
        const int t = (!DIAG && MODE == 0 && std::is_same<CZ, CX>::value && std::is_same<CX, CY>::value)
                          ? tuned_variant(NB, n, nnzb, s, std::is_same<CZ, c64>::value ? CHAFF_C64 : CHAFF_C128)
                          : -1;
        // wide products of mixed precision (the FP64 residual, the FP64 guess) are not in the
        // tuning table: one wave per block row with the block staged in LDS, as the tuned
        // complex64 product at these widths
        const bool wide = !DIAG && NB2 <= 64 && s >= 32;
        variant = t >= 0 ? t : (DIAG ? (s == 1 ? 0 : 1) : wide ? 7 : default_variant(s));
    }
    if (variant == 0) {
        dim3 grid((unsigned)((n * NB + 255) / 256), (unsigned)s);
        hipLaunchKernelGGL((k_spmm_rowq<CZ, CX, CY, MODE, DIAG>), grid, dim3(256), 0, st, row_ptr, col_idx,
                           Z, X, B, Y, n, s);
        CHAFF_LAUNCH_CHECK();
        return CHAFF_OK;
    }
    if constexpr (NB2 > 64) {   // the wave-per-row variants stage a block with one load per lane
        if (variant == 6 || variant == 7) variant = 3;
    }
    if constexpr (NB2 <= 64) if ((variant == 6 || variant == 7) && !DIAG) {
        // S columns per tile, several block rows per wave below 32 columns; 7 = XCD-aware order
        const int sw = spmm_tile_width(s) < 4 ? 4 : spmm_tile_width(s);
        // block rows per wave (several independent gather chains per wave at small widths)
        const int64_t nr = sw == 4 ? 4 : sw == 8 ? 2 : sw == 16 ? 4 : 1;
        const int64_t n_grp = (n + nr - 1) / nr;
        const int64_t nblk = variant == 7 ? (n_grp + NXCD - 1) / NXCD * NXCD : n_grp;
        dim3 grid((unsigned)nblk, (unsigned)((s + sw - 1) / sw));
#define CHAFF_WR(SW, NRW)                                                                                   \
    case SW:                                                                                                \
        if (variant == 7)                                                                                   \
            hipLaunchKernelGGL((k_spmm_wave_row<CZ, CX, CY, MODE, SW, NRW, true>), grid, dim3(64), 0, st,   \
                               row_ptr, col_idx, Z, X, B, Y, n, s);                                         \
        else                                                                                                \
            hipLaunchKernelGGL((k_spmm_wave_row<CZ, CX, CY, MODE, SW, NRW, false>), grid, dim3(64), 0, st,  \
                               row_ptr, col_idx, Z, X, B, Y, n, s);                                         \
        break;
        switch (sw) {
            CHAFF_WR(4, 4) CHAFF_WR(8, 2) CHAFF_WR(16, 4) CHAFF_WR(32, 1) CHAFF_WR(64, 1)
            default: return fail(CHAFF_EINVAL, "bad tile width");
        }
#undef CHAFF_WR
        CHAFF_LAUNCH_CHECK();
        return CHAFF_OK;
    }
    if (variant == 5 && !DIAG) {
        const int sc = s <= 1 ? 1 : s <= 2 ? 2 : s <= 4 ? 4 : s <= 8 ? 8 : 16;
        dim3 grid((unsigned)((n * NB + 255) / 256), (unsigned)((s + sc - 1) / sc));
        const bool vec = std::is_same<CX, c64>::value && (s % 2 == 0) && sc >= 2 &&
                         (reinterpret_cast<uintptr_t>(X) & 15) == 0;
#define CHAFF_RQM(SC)                                                                                        \
    case SC:                                                                                                 \
        if (vec)                                                                                             \
            hipLaunchKernelGGL((k_spmm_rowq_multi<CZ, CX, CY, MODE, SC, true>), grid, dim3(256), 0, st, row_ptr, \
                               col_idx, Z, X, B, Y, n, s);                                                  \
        else                                                                                                 \
            hipLaunchKernelGGL((k_spmm_rowq_multi<CZ, CX, CY, MODE, SC, false>), grid, dim3(256), 0, st,     \
                               row_ptr, col_idx, Z, X, B, Y, n, s);                                          \
        break;
        switch (sc) {
            CHAFF_RQM(1) CHAFF_RQM(2) CHAFF_RQM(4) CHAFF_RQM(8) CHAFF_RQM(16)
            default: return fail(CHAFF_EINVAL, "bad column count");
        }
#undef CHAFF_RQM
        CHAFF_LAUNCH_CHECK();
        return CHAFF_OK;
    }
    int w = spmm_tile_width(s);
    if ((variant == 2 || variant == 4) && w > 1) w >>= 1;
    const unsigned ty = (unsigned)((s + w - 1) / w);
    if (!DIAG && (variant == 3 || variant == 4)) {
        const int64_t row_tiles = (n + (256 / w) - 1) / (256 / w);
        const int64_t per_xcd = (row_tiles + NXCD - 1) / NXCD;
        const unsigned nblk = (unsigned)(per_xcd * NXCD * ty);
#define CHAFF_XCD(W)                                                                                  \
    case W:                                                                                           \
        hipLaunchKernelGGL((k_spmm_xcd<CZ, CX, CY, MODE, W>), dim3(nblk), dim3(256), 0, st, row_ptr,  \
                           col_idx, Z, X, B, Y, n, s, row_tiles, (int)ty);                            \
        break;
        switch (w) {
            CHAFF_XCD(1) CHAFF_XCD(2) CHAFF_XCD(4) CHAFF_XCD(8) CHAFF_XCD(16) CHAFF_XCD(32) CHAFF_XCD(64)
            default: return fail(CHAFF_EINVAL, "bad tile width");
        }
#undef CHAFF_XCD
        CHAFF_LAUNCH_CHECK();
        return CHAFF_OK;
    }
#define CHAFF_TILE(W)                                                                                    \
    case W: {                                                                                            \
        dim3 grid((unsigned)((n + (256 / W) - 1) / (256 / W)), ty);                                      \
        hipLaunchKernelGGL((k_spmm_tile<CZ, CX, CY, MODE, DIAG, W>), grid, dim3(256), 0, st, row_ptr,    \
                           col_idx, Z, X, B, Y, n, s);                                                   \
        break;                                                                                           \
    }
    switch (w) {
        CHAFF_TILE(1) CHAFF_TILE(2) CHAFF_TILE(4) CHAFF_TILE(8) CHAFF_TILE(16) CHAFF_TILE(32) CHAFF_TILE(64)
        default: return fail(CHAFF_EINVAL, "bad tile width");
    }
#undef CHAFF_TILE
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status spmm_public(Cloud* c, chaff_prec prec, const void* Z, const void* X, void* Y, int64_t s,
                         int variant, hipStream_t st) {
    if (prec == CHAFF_C64)
        return spmm_launch<c64, c64, c64, 0, false>(c->row_ptr, c->col_idx, (const c64*)Z, (const c64*)X,
                                                    nullptr, (c64*)Y, c->n, c->nnzb, s, variant, st);
    return spmm_launch<c128, c128, c128, 0, false>(c->row_ptr, c->col_idx, (const c128*)Z, (const c128*)X,
                                                   nullptr, (c128*)Y, c->n, c->nnzb, s, variant, st);
}

// ------------------------------------------------------------------ excitation (FP64)

__device__ __forceinline__ double sinc(double x) {
    return fabs(x) < 1e-4 ? 1.0 - x * x / 6.0 : sin(x) / x;
}

// U[i*7+q][r] (internal wire i) or, with `perm`, at caller row perm[i].
__global__ void k_excitation(const Wire* __restrict__ wires, const int32_t* __restrict__ perm, int64_t n,
                             const double* __restrict__ k_hat, const double* __restrict__ e_hat,
                             int64_t s, double k, c128* __restrict__ U, c64* __restrict__ U32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * s) return;
    const int64_t i = t / s, r = t - (t / s) * s;
    const Wire w = wires[i];
    const double kx = k_hat[3 * r], ky = k_hat[3 * r + 1], kz = k_hat[3 * r + 2];
    const double ex = e_hat[3 * r], ey = e_hat[3 * r + 1], ez = e_hat[3 * r + 2];
    const double tp = w.tx * ex + w.ty * ey + w.tz * ez;
    const double beta = k * (kx * w.tx + ky * w.ty + kz * w.tz);
    const double ph0 = k * (kx * w.cx + ky * w.cy + kz * w.cz);
    const double D = w.len / NSEG;
    const double sc = sinc(0.5 * beta * D);
    const double env = tp * D * sc * sc;
    const int64_t row = perm ? (int64_t)perm[i] : i;
    for (int q = 0; q < NB; ++q) {
        const double sq = -0.5 * w.len + (q + 1) * D;
        double sn, cs;
        sincos(ph0 + beta * sq, &sn, &cs);
        U[(row * NB + q) * s + r] = c128{env * cs, -env * sn};
        if (U32) U32[(row * NB + q) * s + r] = c64{(float)(env * cs), (float)(-env * sn)};
    }
}

// x (FP64) = x32 (FP32), exactly
__global__ void k_widen(const c64* __restrict__ x32, int64_t n, c128* __restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) x[t] = c128{(double)x32[t].re, (double)x32[t].im};
}

// ------------------------------------------------------------------ row-chunk reductions

struct Chunk {
    int64_t w0, w1;      // wire range (internal order), within one cloud
    int32_t cloud;
    int32_t cl0;         // solver chunks: cluster that starts at w0 (chunks are cluster-aligned)
};

constexpr int RB = 256;  // threads per reduction block
constexpr int GV = 8;    // basis vectors per dot group

// Per-thread mapping inside a chunk: ST columns, 256/ST rows per pass.
struct RowMap {
    int st, rsub, r;
};
__device__ __forceinline__ RowMap rowmap(int st) {
    RowMap m;
    m.st = st;
    m.rsub = threadIdx.x / st;
    m.r = blockIdx.y * st + threadIdx.x % st;
    return m;
}

// Reduce acc over the threads sharing a column; lane ST-strided tree in LDS.
__device__ __forceinline__ c128 block_col_reduce(c128 v, int st, c128* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int stride = RB / 2; stride >= st; stride >>= 1) {
        if (threadIdx.x < stride) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + stride]);
        __syncthreads();
    }
    c128 out = red[threadIdx.x % st];
    __syncthreads();
    return out;
}

// part[chunk][slot][s] += dots of V_i (i in [i0, i0+ng)) with W over the chunk
template <typename C>
__global__ __launch_bounds__(RB) void k_dots(const Chunk* __restrict__ chunks, const C* __restrict__ V,
                                             int64_t vstride, int i0, int ng, const C* __restrict__ W,
                                             int64_t s, int st, c128* __restrict__ part, int nslot) {
    __shared__ c128 red[RB];
    const Chunk ch = chunks[blockIdx.x];
    const RowMap m = rowmap(st);
    c128 acc[GV];
#pragma unroll
    for (int g = 0; g < GV; ++g) acc[g] = {0, 0};
    if (m.r < s) {
        for (int64_t row = ch.w0 * NB + m.rsub; row < ch.w1 * NB; row += RB / st) {
            const int64_t o = row * s + m.r;
            c128 w = ccast<c128>(W[o]);
#pragma unroll
            for (int g = 0; g < GV; ++g)
                if (g < ng) cfma_conj(acc[g], ccast<c128>(V[(int64_t)(i0 + g) * vstride + o]), w);
        }
    }
    for (int g = 0; g < ng; ++g) {
        c128 v = block_col_reduce(acc[g], st, red);
        if (threadIdx.x < st && m.r < s) part[((int64_t)blockIdx.x * nslot + i0 + g) * s + m.r] = v;
    }
}

// W -= sum_i V_i h[i][cloud][r]  (i < nv); optional squared norm of the result into slot `nslot_norm`
template <typename C, bool NORM>
__global__ __launch_bounds__(RB) void k_update(const Chunk* __restrict__ chunks, const C* __restrict__ V,
                                               int64_t vstride, int nv, const c128* __restrict__ h,
                                               int n_clouds, C* __restrict__ W, int64_t s, int st,
                                               c128* __restrict__ part, int nslot, int slot_norm) {
    using R = typename real_of<C>::type;
    __shared__ c128 red[RB];
    const Chunk ch = chunks[blockIdx.x];
    const RowMap m = rowmap(st);
    c128 acc = {0, 0};
    if (m.r < s) {
        const int64_t hsys = (int64_t)ch.cloud * s + m.r;
        const int64_t hst = (int64_t)n_clouds * s;
        for (int64_t row = ch.w0 * NB + m.rsub; row < ch.w1 * NB; row += RB / st) {
            const int64_t o = row * s + m.r;
            cplx<R> w = W[o];
            for (int i = 0; i < nv; ++i) {
                cplx<R> hc = ccast<cplx<R>>(h[i * hst + hsys]);
                cplx<R> v = V[(int64_t)i * vstride + o];
                cfma(w, cmk<R>(-v.re, -v.im), hc);
            }
            W[o] = w;
            if (NORM) acc.re += (double)w.re * w.re + (double)w.im * w.im;
        }
    }
    if (NORM) {
        c128 v = block_col_reduce(acc, st, red);
        if (threadIdx.x < st && m.r < s) part[((int64_t)blockIdx.x * nslot + slot_norm) * s + m.r] = v;
    }
}

// squared norms of a vector block into slot
template <typename C>
__global__ __launch_bounds__(RB) void k_norm2(const Chunk* __restrict__ chunks, const C* __restrict__ W,
                                              int64_t s, int st, c128* __restrict__ part, int nslot, int slot) {
    __shared__ c128 red[RB];
    const Chunk ch = chunks[blockIdx.x];
    const RowMap m = rowmap(st);
    c128 acc = {0, 0};
    if (m.r < s) {
        for (int64_t row = ch.w0 * NB + m.rsub; row < ch.w1 * NB; row += RB / st) {
            c128 w = ccast<c128>(W[row * s + m.r]);
            acc.re += w.re * w.re + w.im * w.im;
        }
    }
    c128 v = block_col_reduce(acc, st, red);
    if (threadIdx.x < st && m.r < s) part[((int64_t)blockIdx.x * nslot + slot) * s + m.r] = v;
}

// out[rel][g][r] = sum over k in [off[g], off[g+1]) of in[k*ch_stride + (slot0+rel)*slot_stride + r].
// One 1024-thread block per (rel, g, 64-column tile): wave w sums k = off[g]+w,
// +16, ... (coalesced over the columns), then the 16 wave sums are added in
// wave order.  Fixed order throughout, so the result is reproducible.
constexpr int CS_WAVES = 16;
__global__ __launch_bounds__(64 * CS_WAVES) void k_group_sum(const c128* __restrict__ in, int64_t ch_stride,
                                                             int64_t slot_stride, int slot0,
                                                             const int32_t* __restrict__ off, int n_groups,
                                                             int64_t s, c128* __restrict__ out) {
    __shared__ c128 red[CS_WAVES][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = blockIdx.x % n_groups;
    const int rel = blockIdx.x / n_groups;
    const int64_t r = (int64_t)blockIdx.y * 64 + lane;
    c128 acc = {0, 0};
    if (r < s)
        for (int64_t k = off[g] + w; k < off[g + 1]; k += CS_WAVES)
            acc = cadd(acc, in[k * ch_stride + (int64_t)(slot0 + rel) * slot_stride + r]);
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && r < s) {
        c128 t = red[0][lane];
        for (int k = 1; k < CS_WAVES; ++k) t = cadd(t, red[k][lane]);
        out[((int64_t)rel * n_groups + g) * s + r] = t;
    }
}

static inline void group_sum(const c128* in, int64_t ch_stride, int64_t slot_stride, int slot0, int ns,
                             const int32_t* off, int n_groups, int64_t s, c128* out, hipStream_t st) {
    dim3 grid((unsigned)(ns * n_groups), (unsigned)((s + 63) / 64));
    hipLaunchKernelGGL(k_group_sum, grid, dim3(64 * CS_WAVES), 0, st, in, ch_stride, slot_stride, slot0, off,
                       n_groups, s, out);
}

// out[slot - slot0][cloud][r] = sum over the cloud's chunks of part[chunk][slot][r]
static inline void chunk_sum(const c128* part, const int32_t* cloud_chunk_off, int n_clouds, int nslot, int slot0,
                             int ns, int64_t s, c128* out, hipStream_t st) {
    group_sum(part, (int64_t)nslot * s, s, slot0, ns, cloud_chunk_off, n_clouds, s, out, st);
}

// ------------------------------------------------------------------ per-system GMRES state (FP64)

struct SysState {
    int32_t done;      // 1 once converged or broken down
    int32_t k_used;    // Krylov columns used by the least-squares solve
    double inv_beta;   // 1 / h_{j+1,j} for the next basis vector (0 after breakdown)
    double est;        // current residual estimate relative to the cycle start
    double target;     // stop when est <= target
};

// column j of H from the two CGS passes and ||w||, Givens update, convergence flags
__global__ void k_givens(int64_t nsys, int j, int m, const c128* __restrict__ h1, const c128* __restrict__ h2,
                         const c128* __restrict__ nrm, c128* __restrict__ H, c128* __restrict__ G,
                         double* __restrict__ cs, c128* __restrict__ sn, SysState* __restrict__ sys,
                         int32_t* __restrict__ n_active) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsys) return;
    SysState S = sys[t];
    c128* Hc = H + t * (int64_t)(m + 1) * m;   // H[i][j] at Hc[i*m + j]
    c128* g = G + t * (int64_t)(m + 1);
    double* c_ = cs + t * (int64_t)m;
    c128* s_ = sn + t * (int64_t)m;
    double beta = sqrt(fmax(nrm[t].re, 0.0));
    for (int i = 0; i <= j; ++i) Hc[i * m + j] = cadd(h1[(int64_t)i * nsys + t], h2[(int64_t)i * nsys + t]);
    Hc[(j + 1) * m + j] = c128{beta, 0.0};
    if (S.done) {
        sys[t].inv_beta = 0.0;
        return;
    }
    // previous rotations
    for (int i = 0; i < j; ++i) {
        c128 x = Hc[i * m + j], y = Hc[(i + 1) * m + j];
        c128 nx = cadd(cscale(x, c_[i]), cmul(s_[i], y));
        c128 ny = csub(cscale(y, c_[i]), cmul(c128{s_[i].re, -s_[i].im}, x));
        Hc[i * m + j] = nx;
        Hc[(i + 1) * m + j] = ny;
    }
    c128 a = Hc[j * m + j];
    double aa = sqrt(a.re * a.re + a.im * a.im);
    double cj;
    c128 sj, rr;
    if (beta == 0.0) {
        cj = 1.0; sj = c128{0, 0}; rr = a;
    } else if (aa == 0.0) {
        cj = 0.0; sj = c128{1, 0}; rr = c128{beta, 0};
    } else {
        double tn = sqrt(aa * aa + beta * beta);
        c128 ph = c128{a.re / aa, a.im / aa};
        cj = aa / tn;
        sj = cscale(ph, beta / tn);
        rr = cscale(ph, tn);
    }
    c_[j] = cj;
    s_[j] = sj;
    Hc[j * m + j] = rr;
    Hc[(j + 1) * m + j] = c128{0, 0};
    c128 gj = g[j];
    g[j] = cscale(gj, cj);
    g[j + 1] = cmul(c128{-sj.re, sj.im}, gj);
    double est = sqrt(g[j + 1].re * g[j + 1].re + g[j + 1].im * g[j + 1].im);
    S.est = est;
    S.k_used = j + 1;
    const double hscale = sqrt(aa * aa + beta * beta);
    const bool breakdown = !(beta > 1e-14 * hscale) || !isfinite(beta);
    S.inv_beta = breakdown ? 0.0 : 1.0 / beta;
    if (est <= S.target || breakdown || j + 1 >= m) S.done = 1;
    sys[t] = S;
    if (!S.done) atomicAdd(n_active, 1);
}

// y = R^{-1} g over the first k_used columns, scaled by the cycle's residual norm
__global__ void k_lsq(int64_t nsys, int m, const c128* __restrict__ H, const c128* __restrict__ G,
                      const SysState* __restrict__ sys, const double* __restrict__ rnorm,
                      c128* __restrict__ Y, int nv_max) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsys) return;
    const c128* Hc = H + t * (int64_t)(m + 1) * m;
    const c128* g = G + t * (int64_t)(m + 1);
    const int k = sys[t].k_used;
    c128 y[256];
    for (int i = k - 1; i >= 0; --i) {
        c128 acc = g[i];
        for (int l = i + 1; l < k; ++l) acc = csub(acc, cmul(Hc[i * m + l], y[l]));
        c128 d = Hc[i * m + i];
        double dd = d.re * d.re + d.im * d.im;
        y[i] = dd > 0 ? cmul(acc, c128{d.re / dd, -d.im / dd}) : c128{0, 0};
    }
    const double sc = rnorm[t];
    for (int i = 0; i < nv_max; ++i) Y[(int64_t)i * nsys + t] = i < k ? cscale(y[i], sc) : c128{0, 0};
}

// elementwise helpers -----------------------------------------------------------

// V0 = R * (1/||r||) cast to C; zero for inactive systems
template <typename C>
__global__ void k_start_vector(const c128* __restrict__ Rv, const int32_t* __restrict__ wire_cloud,
                               const double* __restrict__ inv_rn, int n_clouds, int64_t n_rows, int64_t s,
                               C* __restrict__ V0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s) return;
    const int64_t row = t / s, r = t - (t / s) * s;
    const int c = wire_cloud[row / NB];
    const double f = inv_rn[(int64_t)c * s + r];
    V0[t] = ccast<C>(cscale(Rv[t], f));
}

// Vnext = W * inv_beta(system)
template <typename C>
__global__ void k_scale_next(const C* __restrict__ W, const int32_t* __restrict__ wire_cloud,
                             const SysState* __restrict__ sys, int64_t n_rows, int64_t s, C* __restrict__ Vn) {
    using R = typename real_of<C>::type;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s) return;
    const int64_t row = t / s, r = t - (t / s) * s;
    const int c = wire_cloud[row / NB];
    const R f = (R)sys[(int64_t)c * s + r].inv_beta;
    Vn[t] = cscale(W[t], f);
}

// T = sum_{i<nv} V_i Y_i(system)
template <typename C>
__global__ void k_combine(const C* __restrict__ V, int64_t vstride, int nv, const c128* __restrict__ Y,
                          const int32_t* __restrict__ wire_cloud, int n_clouds, int64_t n_rows, int64_t s,
                          C* __restrict__ T) {
    using R = typename real_of<C>::type;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s) return;
    const int64_t row = t / s, r = t - (t / s) * s;
    const int64_t sysi = (int64_t)wire_cloud[row / NB] * s + r;
    const int64_t nsys = (int64_t)n_clouds * s;
    cplx<R> acc = {0, 0};
    for (int i = 0; i < nv; ++i) cfma(acc, V[(int64_t)i * vstride + t], ccast<cplx<R>>(Y[(int64_t)i * nsys + sysi]));
    T[t] = acc;
}

// caller <-> internal permutation of [N*7][s] complex double blocks
__global__ void k_permute_rows(const c128* __restrict__ src, const int32_t* __restrict__ map, int64_t n,
                               int64_t s, c128* __restrict__ dst, int to_caller) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * NB * s) return;
    const int64_t row = t / s, r = t - (t / s) * s;
    const int64_t i = row / NB, q = row - (row / NB) * NB;
    // to_caller: dst[perm[i]] = src[i]  (map = perm);  else dst[i] = src[perm[i]]
    const int64_t p = map[i];
    if (to_caller) dst[(p * NB + q) * s + r] = src[t];
    else dst[t] = src[(p * NB + q) * s + r];
}

__global__ void k_copy_c128(const c128* __restrict__ a, int64_t n, c128* __restrict__ b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = a[t];
}
__global__ void k_zero_bytes(uint32_t* __restrict__ a, int64_t nwords) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nwords;
         t += (int64_t)gridDim.x * blockDim.x)
        a[t] = 0u;
}


// ------------------------------------------------------------------ COCG (complex symmetric CG)
// Z = Z^T exactly (each unique pair is filled once and stored twice, self
// blocks are symmetric by construction) and the block-Jacobi inverse is
// complex symmetric too, so the preconditioned conjugate-orthogonal CG
// recurrence (bilinear form a^T b, no conjugation) applies: six vectors, no
// restarts, one sparse product per step.

struct CgState {
    double rho, rho_im;             // r^T z of the current step
    double rho_prev, rho_prev_im;   // r^T z of the previous step
    double alpha_re, alpha_im;
    double beta_re, beta_im;
    double rnorm;                   // recursive ||r|| (in units of the run's scale)
    double target;                  // freeze once rnorm <= target
    double ckpt;                    // end the cycle once every system is below its checkpoint
    int32_t done;
    int32_t pad;
};

// alpha = rho / (p^T q)
__global__ void k_cg_alpha(int64_t nsys, const c128* __restrict__ pq, CgState* __restrict__ cg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsys) return;
    CgState S = cg[t];
    const c128 d = pq[t];
    const double dd = d.re * d.re + d.im * d.im;
    if (S.done || !(dd > 0.0) || !isfinite(dd)) {
        S.alpha_re = S.alpha_im = 0.0;
        S.done = 1;
    } else {
        const c128 rho = {S.rho, S.rho_im};
        const c128 a = cmul(rho, c128{d.re / dd, -d.im / dd});
        S.alpha_re = a.re;
        S.alpha_im = a.im;
    }
    cg[t] = S;
}


// Compaction flush: x64 += scale * (xc + alpha p), i.e. the deferred x update of
// the last step followed by the flush of the accumulated correction, in one
// pass (the same roundings as applying them one after the other).
template <typename C>
__global__ void k_cg_flush(const int32_t* __restrict__ wire_cloud, const CgState* __restrict__ cg,
                           const double* __restrict__ scale, const int32_t* __restrict__ colmap, int64_t n_rows,
                           int64_t s_cur, int64_t s_full, const C* __restrict__ p, const C* __restrict__ xc,
                           c128* __restrict__ x) {
    using R = typename real_of<C>::type;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s_cur) return;
    const int64_t row = t / s_cur, rr = t - (t / s_cur) * s_cur;
    const int64_t cl = wire_cloud[row / NB];
    const CgState& S = cg[cl * s_cur + rr];
    cplx<R> xv = xc ? xc[t] : cplx<R>{0, 0};   // no xc: nothing accumulated yet this cycle
    cfma(xv, cplx<R>{(R)S.alpha_re, (R)S.alpha_im}, p[t]);
    const int64_t col = colmap[rr];
    const double f = scale[cl * s_full + col];
    const c128 v = ccast<c128>(xv);
    c128& xo = x[row * s_full + col];
    xo = c128{xo.re + f * v.re, xo.im + f * v.im};
}

// dst[row][j] = src[row][keep[j]] (column compaction of a row-major [rows][s] block)
template <typename C>
__global__ void k_gather_cols(const C* __restrict__ src, int64_t n_rows, int64_t s_src,
                              const int32_t* __restrict__ keep, int64_t s_dst, C* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s_dst) return;
    const int64_t row = t / s_dst, j = t - (t / s_dst) * s_dst;
    dst[t] = src[row * s_src + keep[j]];
}

// V0[row][j] = Rv[row][keep[j]] * inv_rn[cloud][keep[j]]: the start vector of a
// COCG cycle restricted to the columns that still hold a live system
template <typename C>
__global__ void k_start_vector_cols(const c128* __restrict__ Rv, const int32_t* __restrict__ wire_cloud,
                                    const double* __restrict__ inv_rn, int64_t n_rows, int64_t s_full,
                                    const int32_t* __restrict__ keep, int64_t s_new, C* __restrict__ V0) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s_new) return;
    const int64_t row = t / s_new, j = t - (t / s_new) * s_new;
    const int64_t col = keep[j];
    const int c = wire_cloud[row / NB];
    V0[t] = ccast<C>(cscale(Rv[row * s_full + col], inv_rn[(int64_t)c * s_full + col]));
}

template <typename T>
__global__ void k_gather_sys(const T* __restrict__ src, int n_clouds, int64_t s_src, const int32_t* __restrict__ keep,
                             int64_t s_dst, T* __restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_clouds * s_dst) return;
    const int64_t cl = t / s_dst, j = t - (t / s_dst) * s_dst;
    dst[t] = src[cl * s_src + keep[j]];
}

// Fused COCG kernels (chunk-structured so that the bilinear forms reduce per
// cloud in a fixed order).  Thread (rsub, r): RHS column r of wire rows
// i = w0 + rsub, w0 + rsub + 256/ST, ... of the block's chunk.
//
// COCG product q = Z p.  A tile is four block rows of one cloud, one row per
// wave; tiles are walked in XCD-aware order (XCD x takes tiles
// [x T/8, (x+1) T/8) in Morton order, so the neighbour slabs a row gathers
// stay in that XCD's L2).  Each wave stages the 7x7 blocks of its row in its
// own LDS slot with one coalesced load, prefetched one block ahead so the
// HBM latency of the Z stream overlaps the arithmetic; lane (group g, column
// c) applies block columns k = g, g + G, ... (G = 64/S) to RHS column c, and
// the G partial sums are combined with cross-lane adds.  sigma = p^T q is
// reduced per tile in FP64 (tpart[tile][r]); the row's own p is stashed in
// LDS when its diagonal block's slab is gathered (no second read of p, no
// registers held across the loop).  Blocks are applied in ascending column
// order: the rows in flight on an XCD then gather their neighbours' slabs in
// step, and L2 serves them (10.2 GB fetched per C5 launch; starting each row
// after its diagonal, so that the own slab came last, fetched 12.9 GB).  Two
// fixed-order passes then sum tiles per group and groups per cloud.  The
// gathers of p bound the kernel: complex64 tiles ask the compiler for at
// least seven waves per SIMD (the 64-column three-product MFMA tile fits 66
// registers; eight waves spill); complex128 tiles would spill under that
// bound.  Gathering the next block's slab during the current block's MFMAs
// measured no faster at C5 (it costs one wave per SIMD).
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int COCG_TILE_ROWS = RB / 64;
template <typename CZ, typename C, int S>
__global__ __launch_bounds__(RB) __attribute__((amdgpu_waves_per_eu(sizeof(C) == sizeof(c64) && NB == 7 ? 7 : 1)))
void k_cocg_spmm(const Chunk* __restrict__ tiles, int64_t n_tiles, int col_tiles, int xcd_order,
                 const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col_idx, const CZ* __restrict__ Z,
                 const C* __restrict__ P, C* __restrict__ Q, int64_t s, c128* __restrict__ tpart) {
    using R = typename real_of<C>::type;
    constexpr int G = 64 / S;
    constexpr int KK = (NB + G - 1) / G;
    constexpr int ZPL = (NB2 + 63) / 64;
    __shared__ CZ zs[COCG_TILE_ROWS][2][NB2];
    __shared__ cplx<typename real_of<C>::type> pown[COCG_TILE_ROWS][(NB + 64 / S - 1) / (64 / S)][64];
    __shared__ c128 red[RB];
    const int64_t id = blockIdx.x;
    int64_t t, ctile_l;
    if (xcd_order) {
        const int xcd = (int)(id % NXCD);
        const int64_t local = id / NXCD;
        const int64_t per_xcd = (n_tiles + NXCD - 1) / NXCD;
        t = (int64_t)xcd * per_xcd + local / col_tiles;
        ctile_l = local % col_tiles;
    } else {
        t = id / col_tiles;
        ctile_l = id % col_tiles;
    }
    if (t >= n_tiles) return;   // uniform over the block
    const Chunk tl = tiles[t];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int g = lane / S, c = lane % S;
    const int64_t i = tl.w0 + w;
    const int64_t r = ctile_l * S + c;
    const int64_t rc = r < s ? r : 0;
    c128 dot = {0, 0};
    // complex64: the 7x7 block times the slab on the FP32 matrix cores
    // (v_mfma_f32_4x4x1_16b_f32: 16 blocks of 4 lanes, lane l = RHS column
    // l % S of depth group l / S; the 4 lanes of an MFMA block share their
    // group, so each block forms its group's partial sums for 4 columns, and
    // the groups are added by the cross-lane sums below.  Rows 0-3 and 4-7 of
    // the block are two 4-row tiles, row 7 zero.  Three real products per
    // complex one (Gauss's form): the sums a.re x.re, a.im x.im and
    // (a.re + a.im)(x.re + x.im) are accumulated apart and combined at the
    // end, so a depth step takes three MFMAs per tile instead of four; its
    // rounding differs from the four-product form by a few units of the
    // largest partial sum, within the FP32 accuracy the refinement corrects)
    constexpr bool PMFMA = sizeof(C) == sizeof(c64) && sizeof(CZ) == sizeof(c64) && NB == 7;
    static_assert(!PMFMA || S % 4 == 0, "an MFMA block of 4 lanes stays inside one depth group");
    if (i < tl.w1) {   // wave-uniform
        cplx<R> acc[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) acc[q] = {0, 0};
        f32x4_t mr[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        f32x4_t mi[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        f32x4_t ms[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
        // blocks in ascending column order; the row's own p slab is stashed in
        // LDS when its diagonal block is gathered (each lane reads back only
        // what it wrote, so no barrier) for p^T q after the loop
        const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
        // lane l stages entries l, l + 64, ... of each block (ZPL per lane)
        CZ zn[ZPL];
        cplx<R> x[KK];
#pragma unroll
        for (int u = 0; u < ZPL; ++u)
            zn[u] = (lane + 64 * u < NB2 && e0 < e1) ? Z[e0 * NB2 + lane + 64 * u] : CZ{0, 0};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) pown[w][kk][lane] = cplx<R>{0, 0};
        for (int64_t e = e0; e < e1; ++e) {
            const int buf = (int)((e - e0) & 1);
#pragma unroll
            for (int u = 0; u < ZPL; ++u)
                if (lane + 64 * u < NB2) zs[w][buf][lane + 64 * u] = zn[u];
            if (e + 1 < e1) {
#pragma unroll
                for (int u = 0; u < ZPL; ++u)
                    if (lane + 64 * u < NB2) zn[u] = Z[(e + 1) * NB2 + lane + 64 * u];
            }
            const int64_t ce = col_idx[e];
            const C* xb = P + ce * NB * s + rc;
#pragma unroll
            for (int kk = 0; kk < KK; ++kk) {
                const int k = g + kk * G;
                x[kk] = k < NB ? ccast<cplx<R>>(xb[k * s]) : cplx<R>{0, 0};
            }
            if (ce == i) {   // wave-uniform: the diagonal block
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) pown[w][kk][lane] = x[kk];
            }
            // the block written above by this wave's lanes is visible to all of its lanes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if constexpr (PMFMA) {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int k = g + kk * G;
                    const float xs = (float)x[kk].re + (float)x[kk].im;
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        const int row = 4 * t + (lane & 3);
                        const c64 a = (row < NB && k < NB) ? ccast<c64>(zs[w][buf][row * NB + k]) : c64{0.f, 0.f};
                        // three real products per complex one: re = a.re x.re - a.im x.im,
                        // im = (a.re + a.im)(x.re + x.im) - a.re x.re - a.im x.im
                        mr[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.re, (float)x[kk].re, mr[t], 0, 0, 0);
                        mi[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.im, (float)x[kk].im, mi[t], 0, 0, 0);
                        ms[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a.re + a.im, xs, ms[t], 0, 0, 0);
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < KK; ++kk) {
                    const int k = g + kk * G;
                    if (k < NB) {
#pragma unroll
                        for (int q = 0; q < NB; ++q) cfma(acc[q], ccast<cplx<R>>(zs[w][buf][q * NB + k]), x[kk]);
                    }
                }
            }
        }
        if constexpr (PMFMA) {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                const float pr = mr[q >> 2][q & 3], pi = mi[q >> 2][q & 3], ps = ms[q >> 2][q & 3];
                acc[q] = cplx<R>{(R)(pr - pi), (R)(ps - pr - pi)};
            }
        }
#pragma unroll
        for (int off = S; off < 64; off <<= 1)
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                acc[q].re += __shfl_xor(acc[q].re, off, 64);
                acc[q].im += __shfl_xor(acc[q].im, off, 64);
            }
        if (r < s) {   // lane g writes rows q = g, g + G, ... and their part of p^T q
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                if (q % G != g) continue;
                const int64_t o = (i * NB + q) * s + r;
                Q[o] = ccast<C>(acc[q]);
                cfma(dot, ccast<c128>(pown[w][q / G][lane]), ccast<c128>(acc[q]));
            }
        }
    }
    // columns: lanes with equal c across waves and groups
    c128 v = block_col_reduce(dot, S, red);
    if (threadIdx.x < S && r < s) tpart[t * s + r] = v;
}

// Search direction and deferred solution update, one pass per step:
//   x += alpha p_old (the step whose residual update ran last; skipped with
//   pend = 0 when that update was already applied), z = P_i r, p = z + beta p_old.
// z is recomputed here from r instead of being stored by the update kernel.
template <typename CZ, typename C, int ST>
__global__ __launch_bounds__(RB) void k_cg_pdir(const Chunk* __restrict__ chunks, const CgState* __restrict__ cg,
                                                const CZ* __restrict__ Pinv, const C* __restrict__ rv,
                                                C* __restrict__ p, C* __restrict__ x, int64_t s, int pend) {
    using R = typename real_of<C>::type;
    const Chunk ch = chunks[blockIdx.x];
    const int rsub = ST == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / ST);
    const int64_t r = (int64_t)blockIdx.y * ST + threadIdx.x % ST;
    if (r >= s) return;
    const CgState& S = cg[(int64_t)ch.cloud * s + r];
    const cplx<R> a = {pend ? (R)S.alpha_re : (R)0, pend ? (R)S.alpha_im : (R)0};
    const cplx<R> b = {(R)S.beta_re, (R)S.beta_im};
    for (int64_t i = ch.w0 + rsub; i < ch.w1; i += RB / ST) {
        cplx<R> res[NB], pv[NB], xv[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const int64_t o = (i * NB + k) * s + r;
            res[k] = rv[o];
            pv[k] = p[o];
            if (pend) xv[k] = x[o];
        }
        const CZ* pb = Pinv + i * NB2;
#pragma unroll
        for (int qq = 0; qq < NB; ++qq) {
            const int64_t o = (i * NB + qq) * s + r;
            cplx<R> z = {0, 0};
#pragma unroll
            for (int k = 0; k < NB; ++k) cfma(z, ccast<cplx<R>>(pb[qq * NB + k]), res[k]);
            if (pend) {
                cfma(xv[qq], a, pv[qq]);
                x[o] = xv[qq];
            }
            cfma(z, b, pv[qq]);
            p[o] = z;
        }
    }
}


// r -= alpha q ; z = P_i r (not stored) ; partial r^T z and ||r||^2
template <typename CZ, typename C, int ST>
__global__ __launch_bounds__(RB) void k_cg_update(const Chunk* __restrict__ chunks, const CgState* __restrict__ cg,
                                                  const CZ* __restrict__ Pinv, const C* __restrict__ q,
                                                  C* __restrict__ rv, int64_t s, c128* __restrict__ part, int nslot,
                                                  int slot0) {
    using R = typename real_of<C>::type;
    __shared__ c128 red[RB];
    const Chunk ch = chunks[blockIdx.x];
    const int rsub = ST == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / ST);
    const int64_t r = (int64_t)blockIdx.y * ST + threadIdx.x % ST;
    c128 rz = {0, 0}, rr = {0, 0};
    if (r < s) {
        const CgState& S = cg[(int64_t)ch.cloud * s + r];
        const cplx<R> na = {-(R)S.alpha_re, -(R)S.alpha_im};
        for (int64_t i = ch.w0 + rsub; i < ch.w1; i += RB / ST) {
            cplx<R> res[NB], qv[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) {   // issue all loads before any arithmetic
                const int64_t o = (i * NB + k) * s + r;
                res[k] = rv[o];
                qv[k] = q[o];
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                cfma(res[k], na, qv[k]);
                rv[(i * NB + k) * s + r] = res[k];
            }
            const CZ* pb = Pinv + i * NB2;
#pragma unroll
            for (int qq = 0; qq < NB; ++qq) {
                cplx<R> acc = {0, 0};
#pragma unroll
                for (int k = 0; k < NB; ++k) cfma(acc, ccast<cplx<R>>(pb[qq * NB + k]), res[k]);
                cfma(rz, ccast<c128>(res[qq]), ccast<c128>(acc));
                rr.re += (double)res[qq].re * res[qq].re + (double)res[qq].im * res[qq].im;
            }
        }
    }
    c128 v = block_col_reduce(rz, ST, red);
    if (threadIdx.x < ST && r < s) part[((int64_t)blockIdx.x * nslot + slot0) * s + r] = v;
    c128 v2 = block_col_reduce(rr, ST, red);
    if (threadIdx.x < ST && r < s) part[((int64_t)blockIdx.x * nslot + slot0 + 1) * s + r] = v2;
}

// r -= alpha q ; partial ||r||^2 (slot0).  The neighbourhood-inverse
// preconditioner forms z = M r and r^T z in a block-sparse product of its own.
// first: the first step of a cycle (alpha = 0), where only the norm is formed
// and q, which holds nothing yet, is not read.
template <typename C, int ST>
__global__ __launch_bounds__(RB) void k_cg_rupd(const Chunk* __restrict__ chunks, const CgState* __restrict__ cg,
                                                const C* __restrict__ q, C* __restrict__ rv, int64_t s,
                                                c128* __restrict__ part, int nslot, int slot0, int first) {
    using R = typename real_of<C>::type;
    __shared__ c128 red[RB];
    const Chunk ch = chunks[blockIdx.x];
    const int rsub = ST == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / ST);
    const int64_t r = (int64_t)blockIdx.y * ST + threadIdx.x % ST;
    c128 rr = {0, 0};
    if (r < s) {
        const CgState& S = cg[(int64_t)ch.cloud * s + r];
        const cplx<R> na = {-(R)S.alpha_re, -(R)S.alpha_im};
        for (int64_t i = ch.w0 + rsub; i < ch.w1; i += RB / ST) {
            cplx<R> res[NB], qv[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) {   // issue all loads before any arithmetic
                const int64_t o = (i * NB + k) * s + r;
                res[k] = rv[o];
                if (!first) qv[k] = q[o];
            }
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (!first) {
                    cfma(res[k], na, qv[k]);
                    rv[(i * NB + k) * s + r] = res[k];
                }
                rr.re += (double)res[k].re * res[k].re + (double)res[k].im * res[k].im;
            }
        }
    }
    c128 v = block_col_reduce(rr, ST, red);
    if (threadIdx.x < ST && r < s) part[((int64_t)blockIdx.x * nslot + slot0) * s + r] = v;
}

// z = M r for one cluster on the FP32 matrix cores (v_mfma_f32_16x16x4_f32,
// full FP32 products and sums): wave w forms the 16-column tile
// [16 w, 16 w + 16) of z for the four 16-row tiles of the block (rows 56-63
// are padding); each 4-deep step of the real form of the complex product
// takes four MFMAs (re re, -im im, re im, im re).  Lane l supplies the
// operand entries (row l % 16, depth l / 16) of the block and (depth l / 16,
// column l % 16) of r, and receives rows 4 (l / 16) + j, j < 4, of column
// l % 16 of each row tile.
__device__ __forceinline__ void cluster_tile_mfma(const c64* __restrict__ ms, const c64* __restrict__ rs,
                                                  int wv, int l, f32x4_t (&zr)[4], f32x4_t (&zi)[4]) {
    const int lr = l & 15, lk = l >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) zr[t] = zi[t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int k0 = 0; k0 < CLR; k0 += 4) {
        const int k = k0 + lk;
        const c64 b = rs[k * 64 + 16 * wv + lr];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int row = 16 * t + lr;
            const c64 a = row < CLR ? ms[row * CLR + k] : c64{0.f, 0.f};
            zr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, b.re, zr[t], 0, 0, 0);
            zr[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a.im, b.im, zr[t], 0, 0, 0);
            zi[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.re, b.im, zi[t], 0, 0, 0);
            zi[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.im, b.re, zi[t], 0, 0, 0);
        }
    }
}

// Cluster preconditioner form of k_cg_update: r -= alpha q, then z = M r per
// cluster (M the cluster's 56 x 56 inverse block), written over q, with the
// partial r^T z and ||r||^2.  One workgroup walks its chunk's clusters; the
// updated residual rows of a cluster are staged in LDS.  Complex64 64-column
// tiles form z on the matrix cores, one 16-column tile per wave; otherwise
// each lane forms rows of z for its columns from LDS reads of the block.
// The MFMA form keeps no rows of the next cluster in flight: it asks the
// compiler for three waves per SIMD (168 registers instead of 236), which
// hides the loads better than the register prefetch of the vector form.
template <typename CZ, typename C, int ST>
constexpr bool cluster_update_mfma() {
    return sizeof(CZ) == sizeof(c64) && sizeof(C) == sizeof(c64) && ST == 64;
}
template <typename CZ, typename C, int ST>
__global__ __launch_bounds__(RB) __attribute__((amdgpu_waves_per_eu(cluster_update_mfma<CZ, C, ST>() ? 3 : 1)))
void k_cg_update_cl(const Chunk* __restrict__ chunks, const CgState* __restrict__ cg, const CZ* __restrict__ Mb,
                    C* qz, C* __restrict__ rv, int64_t s, c128* __restrict__ part, int nslot, int slot0) {
    using R = typename real_of<C>::type;
    // 64-column tiles: two adjacent columns per lane, so every block value
    // read from LDS serves two columns (half the LDS reads per FMA)
    constexpr int CW = ST == 64 ? 2 : 1;
    constexpr int TPC = ST / CW;           // lanes per row group
    constexpr int NSUB = RB / TPC;         // row groups
    constexpr int RPT = (CLR + NSUB - 1) / NSUB;
    constexpr bool FULL = NSUB * RPT == CLR;
    // the block is staged in LDS for complex64 (25 KB); complex128 reads it from memory
    constexpr bool STAGED = sizeof(CZ) == sizeof(c64);
    // complex64 64-column tiles form z = M r on the matrix cores
    constexpr bool MFMA = cluster_update_mfma<CZ, C, ST>();
    static_assert(!MFMA || RB == 4 * 64, "the MFMA form takes four waves of 16 columns each");
    // the residual tile, reused for the final column reduction (RB complex doubles)
    constexpr int RS_N = std::max<int>(CLR * ST, RB * (int)(sizeof(c128) / sizeof(cplx<R>)));
    __shared__ __align__(16) cplx<R> rs[RS_N];
    __shared__ __align__(16) CZ ms[STAGED ? CLR2 : 2];
    const Chunk ch = chunks[blockIdx.x];
    const int col = (int)(threadIdx.x % TPC) * CW;
    const int rsub = (TPC == 64) ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / TPC);
    const int64_t r0 = (int64_t)blockIdx.y * ST + col;
    bool live[CW];
    int64_t rc[CW];
    cplx<R> na[CW];
    c128 rz[CW], rr[CW];
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) {
        live[cc] = r0 + cc < s;
        rc[cc] = live[cc] ? r0 + cc : s - 1;   // loads of idle lanes stay inside the vectors
        na[cc] = cplx<R>{0, 0};
        if (live[cc]) {
            const CgState& S = cg[(int64_t)ch.cloud * s + r0 + cc];
            na[cc] = cplx<R>{-(R)S.alpha_re, -(R)S.alpha_im};
        }
        rz[cc] = rr[cc] = c128{0, 0};
    }
    // MFMA form: r^T z per column 16 w + (l % 16), summed over the wave's rows
    const int wv = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t zcol = (int)blockIdx.y * ST + 16 * wv + (lane & 15);
    c128 rzm = {0, 0};
    // vector form: the next cluster's residual and q rows are loaded while the
    // current one is multiplied (software pipelining across the chunk's
    // clusters); the MFMA form loads each cluster's rows when it starts it
    cplx<R> res[RPT * CW], qv[RPT * CW];
    auto load_rows = [&](int64_t w_, cplx<R>* res_, cplx<R>* qv_) {
        const int nr_ = (int)std::min<int64_t>(CLW, ch.w1 - w_) * NB;
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int rho = std::min(rsub * RPT + j, nr_ - 1);
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) {
                const int64_t o = (w_ * NB + rho) * s + rc[cc];
                res_[j * CW + cc] = rv[o];
                qv_[j * CW + cc] = qz[o];
            }
        }
    };
    constexpr bool PIPE = !MFMA;
    if (PIPE && ch.w0 < ch.w1) load_rows(ch.w0, res, qv);
    int64_t kc = ch.cl0;
    for (int64_t w = ch.w0; w < ch.w1; w += CLW, ++kc) {
        const int nr = (int)std::min<int64_t>(CLW, ch.w1 - w) * NB;
        const int64_t row0 = w * NB;
        const CZ* mb = Mb + kc * CLR2;
        if (!PIPE) load_rows(w, res, qv);
        if (STAGED) stage_block<CZ, RB>(ms, mb);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int rho = rsub * RPT + j;
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) {
                const bool ok = live[cc] && rho < nr;
                cplx<R> v = res[j * CW + cc];
                cfma(v, na[cc], qv[j * CW + cc]);
                if (!ok) v = cplx<R>{0, 0};
                if (ok) {
                    rv[(row0 + rho) * s + r0 + cc] = v;
                    rr[cc].re += (double)v.re * v.re + (double)v.im * v.im;
                }
                if (FULL || rho < CLR) rs[rho * ST + col + cc] = v;
            }
        }
        __syncthreads();
        if (PIPE && w + CLW < ch.w1) load_rows(w + CLW, res, qv);   // r and q of this cluster live in rs and qz now
        if constexpr (MFMA) {
            f32x4_t zr[4], zi[4];
            cluster_tile_mfma(reinterpret_cast<const c64*>(ms), reinterpret_cast<const c64*>(rs), wv, lane, zr, zi);
            if (zcol < s) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int rho = 16 * t + 4 * (lane >> 4) + j;
                        if (rho < nr) {   // the residual is re-read from its LDS tile
                            const cplx<R> zv = {zr[t][j], zi[t][j]};
                            qz[(row0 + rho) * s + zcol] = zv;
                            cfma(rzm, ccast<c128>(rs[rho * ST + 16 * wv + (lane & 15)]), ccast<c128>(zv));
                        }
                    }
            }
        } else {
            cplx<R> acc[RPT * CW];
            cluster_rows<R, CZ, ST, RPT, FULL, STAGED, CW>(ms, mb, rs, col, rsub, acc);
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int rho = rsub * RPT + j;
#pragma unroll
                for (int cc = 0; cc < CW; ++cc) {
                    if (live[cc] && rho < nr) {   // the residual is re-read from its LDS tile
                        qz[(row0 + rho) * s + r0 + cc] = acc[j * CW + cc];
                        cfma(rz[cc], ccast<c128>(rs[rho * ST + col + cc]), ccast<c128>(acc[j * CW + cc]));
                    }
                }
            }
        }
        __syncthreads();
    }
    // column sums: lanes with equal (lane % TPC) hold the same columns
    c128* red = reinterpret_cast<c128*>(rs);
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) {
        if constexpr (!MFMA) {
            c128 v = block_col_reduce(rz[cc], TPC, red);
            if ((int)threadIdx.x < TPC && live[cc]) part[((int64_t)blockIdx.x * nslot + slot0) * s + r0 + cc] = v;
        }
        c128 v2 = block_col_reduce(rr[cc], TPC, red);
        if ((int)threadIdx.x < TPC && live[cc]) part[((int64_t)blockIdx.x * nslot + slot0 + 1) * s + r0 + cc] = v2;
    }
    if constexpr (MFMA) {   // r^T z: the four row groups of a column sit in lanes l, l + 16, l + 32, l + 48
#pragma unroll
        for (int off = 16; off < 64; off <<= 1) {
            rzm.re += __shfl_xor(rzm.re, off, 64);
            rzm.im += __shfl_xor(rzm.im, off, 64);
        }
        if (lane < 16 && zcol < s) part[((int64_t)blockIdx.x * nslot + slot0) * s + zcol] = rzm;
    }
}

// Form of k_cg_pdir where z was stored by the update (cluster) or by its own
// product (neighbourhood inverse):
//   x += alpha p_old (deferred; skipped with pend = 0; with pend = 2 x holds
//   nothing yet and is written as alpha p_old), p = z + beta p_old (with
//   pfirst, the first step of a cycle, p = z: p_old holds nothing yet).
template <typename C, int ST>
__global__ __launch_bounds__(RB) void k_cg_pdir_z(const Chunk* __restrict__ chunks, const CgState* __restrict__ cg,
                                                  const C* __restrict__ z, C* __restrict__ p, C* __restrict__ x,
                                                  int64_t s, int pend, int pfirst) {
    using R = typename real_of<C>::type;
    const Chunk ch = chunks[blockIdx.x];
    const int rsub = ST == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / ST);
    const int64_t r = (int64_t)blockIdx.y * ST + threadIdx.x % ST;
    if (r >= s) return;
    const CgState& S = cg[(int64_t)ch.cloud * s + r];
    const cplx<R> a = {pend ? (R)S.alpha_re : (R)0, pend ? (R)S.alpha_im : (R)0};
    const cplx<R> b = {(R)S.beta_re, (R)S.beta_im};
    if (pfirst) {
        for (int64_t row = ch.w0 * NB + rsub; row < ch.w1 * NB; row += RB / ST) p[row * s + r] = z[row * s + r];
        return;
    }
    for (int64_t row = ch.w0 * NB + rsub; row < ch.w1 * NB; row += RB / ST) {
        const int64_t o = row * s + r;
        const cplx<R> pv = p[o];
        cplx<R> zv = z[o];
        if (pend) {
            cplx<R> xv = pend == 2 ? cplx<R>{0, 0} : x[o];
            cfma(xv, a, pv);
            x[o] = xv;
        }
        cfma(zv, b, pv);
        p[o] = zv;
    }
}

// After the update: new rho = r^T z, recursive norm; convergence and checkpoint
// flags; beta for p = z + beta p.  mode 0: first step of a run (beta = 0);
// mode 1: ordinary step; mode 2: step right after a residual replacement
// (rho_prev is kept as the denominator).
__global__ void k_cg_step(int64_t nsys, const c128* __restrict__ rz, const c128* __restrict__ rr, int mode,
                          CgState* __restrict__ cg, int32_t* __restrict__ n_active, int32_t* __restrict__ flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsys) return;
    CgState S = cg[t];
    const double rn = sqrt(fmax(rr[t].re, 0.0));
    const c128 rho_new = rz[t];
    if (!S.done) S.rnorm = rn;
    if (!S.done && (rn <= S.target || !isfinite(rn))) S.done = 1;
    const c128 den = (mode == 1) ? c128{S.rho, S.rho_im} : c128{S.rho_prev, S.rho_prev_im};
    const double dd = den.re * den.re + den.im * den.im;
    if (S.done) {   // alpha stays: the deferred x update of this step is still to be applied
        S.beta_re = S.beta_im = 0.0;
    } else if (mode == 0 || !(dd > 0.0)) {
        S.beta_re = S.beta_im = 0.0;
    } else {
        const c128 b = cmul(rho_new, c128{den.re / dd, -den.im / dd});
        S.beta_re = b.re;
        S.beta_im = b.im;
    }
    if (mode == 1) {
        S.rho_prev = S.rho;
        S.rho_prev_im = S.rho_im;
    }
    S.rho = rho_new.re;
    S.rho_im = rho_new.im;
    cg[t] = S;
    const int above = (!S.done && rn > S.ckpt) ? 1 : 0;
    flags[t] = above;
    if (above) atomicAdd(n_active, 1);
}

// start of a cycle: targets, checkpoint, alpha = 0 (the update kernel then only forms z)
__global__ void k_cg_cycle_start(int64_t nsys, const double* __restrict__ target, const double* __restrict__ ckpt,
                                 const int32_t* __restrict__ active, int first, CgState* __restrict__ cg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsys) return;
    CgState S = first ? CgState{} : cg[t];
    S.target = target[t];
    S.ckpt = ckpt[t];
    S.done = active[t] ? 0 : 1;
    S.alpha_re = S.alpha_im = 0.0;
    cg[t] = S;
}

// ------------------------------------------------------------------ host driver

// CHAFF_VERBOSE=1 in the environment prints one line per refinement cycle
// (and the COCG progress every 50 steps)
static const bool g_verbose = [] {
    const char* v = std::getenv("CHAFF_VERBOSE");
    return v && v[0] == '1';
}();

static unsigned blocks_for(int64_t n, int threads = 256) {
    return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads);
}

struct SolveLayout {
    size_t bytes;
    c128 *b, *x, *r;                 // FP64 [rows][s]
    void* V;                         // (m+1) x [rows][s] of C
    void* W;                         // [rows][s] of C
    void* T;                         // [rows][s] of C
    c128* part;                      // [nch][nslot][s]
    c128 *h1, *h2, *nrm, *red;       // [slot][cloud][s]
    c128 *H, *G, *sn, *Y;            // per system
    double *cs, *bn, *rn, *inv_rn;   // per system
    SysState* sys;
    CgState* cg;
    double* target;
    int32_t* active;
    Chunk* chunks;
    int32_t* cloud_chunk_off;
    int32_t* counter;
    Chunk* tiles;              // COCG product tiles
    int32_t* group_tile_off;   // [n_groups+1] tile ranges of the groups
    int32_t* cloud_group_off;  // [n_clouds+1] group ranges of the clouds
    c128* tpart;               // [n_tiles][s]
    c128* gpart;               // [n_groups][s]
    // COCG column compaction: tile set of the narrower width, column maps
    Chunk* ctiles;
    int32_t* cgroup_tile_off;
    int32_t* ccloud_group_off;
    int32_t* colmap;           // [s] current column -> caller RHS column
    int32_t* keep;             // [s] kept columns of a compaction
    CgState* cg2;              // [nsys] staging of the compacted states
};

// Wires per reduction chunk (about 2048 chunks in total): streaming kernels
// reduce per chunk; COCG's product uses its own small tiles (see k_cocg_spmm).
// Wires per solver chunk: a multiple of the cluster width, so that chunks
// starting at a cloud's first wire never split a cluster.
static int64_t chunk_wires(int64_t n, int /*method*/) {
    return (int64_t)align_up((size_t)std::max<int64_t>(32, (n + 2047) / 2048), CLW);
}
constexpr int TILE_GROUP = 256;   // tiles per first-stage group of the sigma reduction

struct SolveShape {
    int64_t n, rows, s, nsys;
    int m, nslot, n_chunks, n_clouds;
    int method, nvec, mg;   // mg: Hessenberg width (GMRES m, COCG 1)
    int64_t n_tiles;        // COCG product tiles (cloud-aligned, tile_w wires)
    int cocg_st, cocg_xcd;  // COCG product: RHS tile width, XCD-aware order
    int n_groups, tile_w;   // tile groups (cloud-aligned, TILE_GROUP tiles)
    size_t csize;
};

static SolveShape solve_shape(const Cloud* c, int m, int64_t s, chaff_prec prec, int method) {
    SolveShape sh;
    sh.method = method;
    const bool cocg = method == CHAFF_COCG || method == CHAFF_COCG_RR;
    sh.mg = cocg ? 1 : m;
    // GMRES: m + 1 basis vectors; GCR: m directions, their m images, the
    // working residual and the correction; COCG: four vectors
    sh.nvec = method == CHAFF_GMRES ? m + 1 : method == CHAFF_GCR ? 2 * m + 2 : 4;
    sh.n = c->n;
    sh.rows = c->n * NB;
    sh.s = s;
    sh.n_clouds = c->n_clouds;
    sh.nsys = (int64_t)c->n_clouds * s;
    sh.m = m;
    sh.nslot = sh.mg + 3;
    const int64_t cw = chunk_wires(c->n, method);
    int64_t nch = 0;
    for (int k = 0; k < c->n_clouds; ++k) {
        int64_t nw = c->cloud_off[k + 1] - c->cloud_off[k];
        nch += (nw + cw - 1) / cw;
    }
    sh.n_chunks = (int)nch;
    sh.n_tiles = 0;
    sh.n_groups = 0;
    sh.cocg_st = cocg_width(s);
    sh.cocg_xcd = 1;
    {   // the COCG product follows the tuned public variant's workgroup order (1, 2, 6: linear)
        int v = tuned_variant(NB, c->n, c->nnzb, s, prec);
        if (v < 0) v = default_variant(s);
        sh.cocg_xcd = (v == 1 || v == 2 || v == 6) ? 0 : 1;
    }
    sh.tile_w = COCG_TILE_ROWS;
    if (cocg) {
        for (int k = 0; k < c->n_clouds; ++k) {
            const int64_t nw = c->cloud_off[k + 1] - c->cloud_off[k];
            const int64_t nt = (nw + sh.tile_w - 1) / sh.tile_w;
            sh.n_tiles += nt;
            sh.n_groups += (int)((nt + TILE_GROUP - 1) / TILE_GROUP);
        }
    }
    sh.csize = prec == CHAFF_C64 ? sizeof(c64) : sizeof(c128);
    return sh;
}

static SolveLayout carve_solve(void* ws, size_t ws_bytes, const SolveShape& sh) {
    Carve cv(ws, ws_bytes);
    SolveLayout L;
    const int64_t vs = sh.rows * sh.s;
    L.b = cv.take<c128>(vs);
    L.x = cv.take<c128>(vs);
    L.r = cv.take<c128>(vs);
    const bool gm = sh.method == CHAFF_GMRES;
    L.V = cv.take<char>((size_t)sh.nvec * vs * sh.csize);
    L.W = gm ? cv.take<char>((size_t)vs * sh.csize) : nullptr;
    L.T = gm ? cv.take<char>((size_t)vs * sh.csize) : nullptr;
    L.part = cv.take<c128>((size_t)std::max(sh.n_chunks, 1) * sh.nslot * sh.s);
    L.h1 = cv.take<c128>((size_t)(sh.mg + 1) * sh.nsys);
    L.h2 = cv.take<c128>((size_t)(sh.mg + 1) * sh.nsys);
    L.nrm = cv.take<c128>((size_t)sh.nsys);
    L.red = cv.take<c128>((size_t)sh.nsys);
    L.H = cv.take<c128>((size_t)sh.nsys * (sh.mg + 1) * sh.mg);
    L.G = cv.take<c128>((size_t)sh.nsys * (sh.mg + 1));
    L.sn = cv.take<c128>((size_t)sh.nsys * sh.mg);
    L.Y = cv.take<c128>((size_t)sh.nsys * (sh.mg + 1));
    L.cs = cv.take<double>((size_t)sh.nsys * sh.mg);
    L.bn = cv.take<double>((size_t)sh.nsys);
    L.rn = cv.take<double>((size_t)sh.nsys);
    L.inv_rn = cv.take<double>((size_t)sh.nsys);
    L.sys = cv.take<SysState>((size_t)sh.nsys);
    L.cg = cv.take<CgState>((size_t)sh.nsys);
    L.target = cv.take<double>((size_t)sh.nsys);
    L.active = cv.take<int32_t>((size_t)sh.nsys);
    L.chunks = cv.take<Chunk>((size_t)std::max(sh.n_chunks, 1));
    L.cloud_chunk_off = cv.take<int32_t>((size_t)sh.n_clouds + 1);
    L.counter = cv.take<int32_t>(64);
    L.tiles = cv.take<Chunk>((size_t)std::max<int64_t>(sh.n_tiles, 1));
    L.group_tile_off = cv.take<int32_t>((size_t)sh.n_groups + 1);
    L.cloud_group_off = cv.take<int32_t>((size_t)sh.n_clouds + 1);
    L.tpart = cv.take<c128>((size_t)std::max<int64_t>(sh.n_tiles, 1) * sh.s);
    L.gpart = cv.take<c128>((size_t)std::max(sh.n_groups, 1) * sh.s);
    // a narrower RHS tile means wider (never more) tiles and groups
    L.ctiles = cv.take<Chunk>((size_t)std::max<int64_t>(sh.n_tiles, 1));
    L.cgroup_tile_off = cv.take<int32_t>((size_t)sh.n_groups + 1);
    L.ccloud_group_off = cv.take<int32_t>((size_t)sh.n_clouds + 1);
    L.colmap = cv.take<int32_t>((size_t)sh.s);
    L.keep = cv.take<int32_t>((size_t)sh.s);
    L.cg2 = cv.take<CgState>((size_t)sh.nsys);
    L.bytes = cv.off + 256;
    return L;
}

size_t solve_workspace_bytes(const Cloud* c, const chaff_solve_opts* o, int64_t s) {
    const int m = o->restart;
    SolveShape sh = solve_shape(c, m, s, (chaff_prec)o->prec, o->method);
    return carve_solve(nullptr, 0, sh).bytes;
}

// COCG product tiles of tile_w wires (cloud-aligned) and their groups of
// TILE_GROUP tiles (cloud-aligned): tl, group -> first tile (gto, + end),
// cloud -> first group (cgo, + end).
static void build_tiles(const Cloud* c, int64_t tile_w, std::vector<Chunk>& tl, std::vector<int32_t>& gto,
                        std::vector<int32_t>& cgo) {
    tl.clear();
    gto.clear();
    cgo.assign(c->n_clouds + 1, 0);
    for (int k = 0; k < c->n_clouds; ++k) {
        cgo[k] = (int32_t)gto.size();
        const int64_t t0 = (int64_t)tl.size();
        for (int64_t w0 = c->cloud_off[k]; w0 < c->cloud_off[k + 1]; w0 += tile_w)
            tl.push_back(Chunk{w0, std::min<int64_t>(w0 + tile_w, c->cloud_off[k + 1]), k, 0});
        for (int64_t g = t0; g < (int64_t)tl.size(); g += TILE_GROUP) gto.push_back((int32_t)g);
    }
    cgo[c->n_clouds] = (int32_t)gto.size();
    gto.push_back((int32_t)tl.size());
}

// per-system squared norms of an FP64 block into host vector (sync)
template <typename C>
static chaff_status norms_to(const SolveShape& sh, SolveLayout& L, const C* v, c128* dst, hipStream_t st) {
    const int wst = spmm_tile_width(sh.s);
    dim3 grid(sh.n_chunks, (unsigned)((sh.s + wst - 1) / wst));
    if (sh.n_chunks > 0) {
        hipLaunchKernelGGL((k_norm2<C>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, v, sh.s, wst, L.part,
                           sh.nslot, 0);
        CHAFF_LAUNCH_CHECK();
    }
    chunk_sum((const c128*)L.part,
                       (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, 0, 1, sh.s, dst, st);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}


template <typename CZ, typename C, int ST>
static void launch_cg_update(const SolveShape& sh, SolveLayout& L, const CZ* Pinv, const C* q, C* r,
                             hipStream_t st) {
    const dim3 grid(sh.n_chunks, (unsigned)((sh.s + ST - 1) / ST));
    hipLaunchKernelGGL((k_cg_update<CZ, C, ST>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const CgState*)L.cg,
                       Pinv, q, r, sh.s, L.part, sh.nslot, 0);
}
template <typename CZ, typename C, int ST>
static void launch_cg_pdir(const SolveShape& sh, SolveLayout& L, const CZ* Pinv, const C* r, C* p, C* x, int pend,
                           hipStream_t st) {
    const dim3 grid(sh.n_chunks, (unsigned)((sh.s + ST - 1) / ST));
    hipLaunchKernelGGL((k_cg_pdir<CZ, C, ST>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const CgState*)L.cg,
                       Pinv, r, p, x, sh.s, pend);
}
template <typename C, int ST>
static void launch_cg_rupd(const SolveShape& sh, SolveLayout& L, const C* q, C* r, bool first, hipStream_t st) {
    const dim3 grid(sh.n_chunks, (unsigned)((sh.s + ST - 1) / ST));
    hipLaunchKernelGGL((k_cg_rupd<C, ST>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const CgState*)L.cg, q, r,
                       sh.s, L.part, sh.nslot, 1, first ? 1 : 0);
}
template <typename CZ, typename C, int ST>
static void launch_cg_update_cl(const SolveShape& sh, SolveLayout& L, const CZ* Mb, C* qz, C* r, hipStream_t st) {
    if constexpr (NB == 7) {   // clusters of 8 wires x 7 unknowns (solve_impl refuses them otherwise)
        const dim3 grid(sh.n_chunks, (unsigned)((sh.s + ST - 1) / ST));
        hipLaunchKernelGGL((k_cg_update_cl<CZ, C, ST>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks,
                           (const CgState*)L.cg, Mb, qz, r, sh.s, L.part, sh.nslot, 0);
    }
}
template <typename C, int ST>
static void launch_cg_pdir_z(const SolveShape& sh, SolveLayout& L, const C* z, C* p, C* x, int pend, bool pfirst,
                             hipStream_t st) {
    const dim3 grid(sh.n_chunks, (unsigned)((sh.s + ST - 1) / ST));
    hipLaunchKernelGGL((k_cg_pdir_z<C, ST>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const CgState*)L.cg,
                       z, p, x, sh.s, pend, pfirst ? 1 : 0);
}
template <typename CZ, typename C, int ST>
static void launch_cocg_spmm(const Cloud* c, const SolveShape& sh, SolveLayout& L, const CZ* Z, const C* p, C* q,
                             hipStream_t st) {
    const int ct = (int)((sh.s + ST - 1) / ST);
    const int64_t per_xcd = (sh.n_tiles + NXCD - 1) / NXCD;
    const int64_t nblk = sh.cocg_xcd ? per_xcd * NXCD * ct : sh.n_tiles * ct;
    hipLaunchKernelGGL((k_cocg_spmm<CZ, C, ST>), dim3((unsigned)nblk), dim3(RB), 0, st,
                       (const Chunk*)L.tiles, sh.n_tiles, ct, sh.cocg_xcd, (const int64_t*)c->row_ptr,
                       (const int32_t*)c->col_idx, Z, p, q, sh.s, L.tpart);
}

static chaff_status cocg_narrow_shape(const Cloud* c, SolveShape& cs, SolveLayout& Lc, const SolveLayout& L,
                                      std::vector<int32_t>& colmap, const std::vector<int32_t>& keep,
                                      hipStream_t st);

// Column compaction inside a COCG cycle: once at most half of the current
// RHS tile width still has a system above its checkpoint, the finished
// columns are dropped -- their accumulated corrections are flushed into the
// FP64 solution, the live columns of r, z, p and their recurrence states are
// packed into a narrower row-major block, and the product switches to the
// matching tile width.  Systems below their checkpoint would only keep
// improving, so dropping them does not change what the cycle guarantees.
template <typename C>
static chaff_status cocg_compact(const Cloud* c, SolveShape& cs, SolveLayout& Lc, const SolveLayout& L,
                                 std::vector<int32_t>& colmap, const std::vector<int32_t>& keep, int64_t s_full,
                                 C*& xc, C*& r, C*& p, C*& q, bool q_live, bool xc_valid, bool p_valid,
                                 hipStream_t st) {
    const int64_t rows = cs.rows, s_old = cs.s, s_new = (int64_t)keep.size();
    ProfScope ps("cocg_compact", st,
                 (double)rows * s_old * (2.0 * sizeof(C) + 2.0 * sizeof(c128)) +
                     (double)rows * (s_old + s_new) * sizeof(C) * (q_live ? 3 : 2) + (double)rows * s_new * sizeof(C));
    // flush every column's correction (with the deferred update of the last step) into the FP64 solution;
    // before the first search direction there is nothing to flush (alpha is still 0)
    if (p_valid) {
        hipLaunchKernelGGL((k_cg_flush<C>), dim3(blocks_for(rows * s_old)), dim3(256), 0, st,
                           (const int32_t*)c->wire_cloud, (const CgState*)L.cg, (const double*)L.rn,
                           (const int32_t*)L.colmap, rows, s_old, s_full, (const C*)p,
                           xc_valid ? (const C*)xc : (const C*)nullptr, L.x);
        CHAFF_LAUNCH_CHECK();
    }
    CHAFF_HIP(hipMemcpyAsync(L.keep, keep.data(), s_new * sizeof(int32_t), hipMemcpyHostToDevice, st));
    // the live columns move into the buffer freed before them (xc, then r, then p): no copies back
    C* const bx = xc;
    C* const br = r;
    C* const bp = p;
    C* const bq = q;
    hipLaunchKernelGGL((k_gather_cols<C>), dim3(blocks_for(rows * s_new)), dim3(256), 0, st, (const C*)br, rows, s_old,
                       (const int32_t*)L.keep, s_new, bx);
    CHAFF_LAUNCH_CHECK();
    if (p_valid) {
        hipLaunchKernelGGL((k_gather_cols<C>), dim3(blocks_for(rows * s_new)), dim3(256), 0, st, (const C*)bp, rows,
                           s_old, (const int32_t*)L.keep, s_new, br);
        CHAFF_LAUNCH_CHECK();
    }
    r = bx;
    p = br;
    if (q_live) {   // z kept in q between the update and the direction pass
        hipLaunchKernelGGL((k_gather_cols<C>), dim3(blocks_for(rows * s_new)), dim3(256), 0, st, (const C*)bq, rows,
                           s_old, (const int32_t*)L.keep, s_new, bp);
        CHAFF_LAUNCH_CHECK();
        q = bp;
        xc = bq;
    } else {        // q is rebuilt by the next product
        q = bp;
        xc = bq;
    }
    {   // the new correction starts at zero
        const int64_t words = rows * s_new * (int64_t)sizeof(C) / 4;
        hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(words)), dim3(256), 0, st, (uint32_t*)xc, words);
        CHAFF_LAUNCH_CHECK();
    }
    return cocg_narrow_shape(c, cs, Lc, L, colmap, keep, st);
}

// The recurrence states, the column map and the tile set of a COCG cycle
// switch to the columns in keep (uploaded to L.keep by the caller).
static chaff_status cocg_narrow_shape(const Cloud* c, SolveShape& cs, SolveLayout& Lc, const SolveLayout& L,
                                      std::vector<int32_t>& colmap, const std::vector<int32_t>& keep,
                                      hipStream_t st) {
    const int64_t s_old = cs.s, s_new = (int64_t)keep.size();
    hipLaunchKernelGGL((k_gather_sys<CgState>), dim3(blocks_for((int64_t)cs.n_clouds * s_new, 64)), dim3(64), 0, st,
                       (const CgState*)L.cg, cs.n_clouds, s_old, (const int32_t*)L.keep, s_new, L.cg2);
    CHAFF_LAUNCH_CHECK();
    CHAFF_HIP(hipMemcpyAsync(L.cg, L.cg2, (size_t)cs.n_clouds * s_new * sizeof(CgState), hipMemcpyDeviceToDevice, st));
    std::vector<int32_t> cm(s_new);
    for (int64_t j = 0; j < s_new; ++j) cm[j] = colmap[keep[j]];
    colmap = cm;
    CHAFF_HIP(hipMemcpyAsync(L.colmap, colmap.data(), s_new * sizeof(int32_t), hipMemcpyHostToDevice, st));
    cs.s = s_new;
    cs.nsys = (int64_t)cs.n_clouds * s_new;
    cs.cocg_st = cocg_width(s_new);
    cs.tile_w = COCG_TILE_ROWS;
    std::vector<Chunk> tl;
    std::vector<int32_t> gto, cgo;
    build_tiles(c, cs.tile_w, tl, gto, cgo);
    cs.n_tiles = (int64_t)tl.size();
    cs.n_groups = (int)gto.size() - 1;
    if (!tl.empty())
        CHAFF_HIP(hipMemcpyAsync(L.ctiles, tl.data(), tl.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
    CHAFF_HIP(hipMemcpyAsync(L.cgroup_tile_off, gto.data(), gto.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    CHAFF_HIP(hipMemcpyAsync(L.ccloud_group_off, cgo.data(), cgo.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                             st));
    Lc.tiles = L.ctiles;
    Lc.group_tile_off = L.cgroup_tile_off;
    Lc.cloud_group_off = L.ccloud_group_off;
    CHAFF_HIP(hipStreamSynchronize(st));   // host staging vectors leave scope
    return CHAFF_OK;
}

// One COCG refinement cycle.  L.r holds the FP64 true residual; it replaces the
// recursive residual (in units of the run's fixed per-system scale).  With
// CHAFF_COCG the recurrence restarts from it; with CHAFF_COCG_RR the search
// direction p and r^T z carry over from the previous cycle ("reliable
// updates").  The cycle ends once every active system's recursive residual
// fell below its checkpoint (or its final target); then x += scale *
// (accumulated correction).
template <typename C, typename CZ>
static chaff_status cocg_cycle(Cloud* c, const chaff_solve_opts* o, const SolveShape& sh, SolveLayout& L,
                               const CZ* Z, const CZ* Pinv, const std::vector<double>& target,
                               const std::vector<double>& ckpt, const std::vector<int32_t>& act, bool first,
                               int& iters, bool& capped, hipStream_t st) {
    capped = false;
    const int64_t rows = sh.rows, s = sh.s, vs = rows * s, nsys = sh.nsys;
    C* V = static_cast<C*>(L.V);   // [x_c | r | p | q], each with room for [rows][s]
    C* xc = V;
    C* r = V + vs;
    C* p = V + 2 * vs;
    C* q = V + 3 * vs;
    const bool use_rr = o->method == CHAFF_COCG_RR;
    const bool compact = !use_rr && s > 1;
    // cluster preconditioner: z = M r is formed by the update and kept in q
    const bool clus = o->precond == CHAFF_PRECOND_CLUSTER;
    const CZ* Mb = clus ? reinterpret_cast<const CZ*>(reinterpret_cast<const char*>(Pinv) +
                                                      cluster_table_bytes(cluster_count(c)))
                        : nullptr;
    // neighbourhood inverse: Pinv is M on Z's block pattern; z = M r is a product of its own, kept in q
    const bool nbhd = o->precond == CHAFF_PRECOND_NBHD;
    const bool zq = clus || nbhd;   // z lives in q between the update and the direction pass
    SolveShape cs = sh;            // current shape (columns shrink under compaction)
    SolveLayout Lc = L;            // current tile set
    std::vector<int32_t> colmap(s);
    for (int64_t j = 0; j < s; ++j) colmap[j] = (int32_t)j;
    CHAFF_HIP(hipMemcpyAsync(L.colmap, colmap.data(), s * sizeof(int32_t), hipMemcpyHostToDevice, st));
    CHAFF_HIP(hipMemcpyAsync(L.target, target.data(), nsys * sizeof(double), hipMemcpyHostToDevice, st));
    CHAFF_HIP(hipMemcpyAsync(L.h2, ckpt.data(), nsys * sizeof(double), hipMemcpyHostToDevice, st));
    CHAFF_HIP(hipMemcpyAsync(L.active, act.data(), nsys * sizeof(int32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_cg_cycle_start, dim3(blocks_for(nsys, 64)), dim3(64), 0, st, nsys, (const double*)L.target,
                       (const double*)L.h2, (const int32_t*)L.active, first ? 1 : 0, L.cg);
    CHAFF_LAUNCH_CHECK();
    // With the neighbourhood inverse a fresh recurrence skips the passes that
    // only carry zeros: x_c, p and q are not cleared, the first step forms
    // ||r||^2 without the update r -= 0 q, sets p = z without reading p, and
    // the first correction is written as alpha p rather than added to x_c.
    const bool lazy = nbhd && !use_rr;   // (COCG_RR carries p and q into the next cycle)
    bool xc_valid = !lazy, p_valid = !lazy;
    // columns that hold a live system: with at most half a tile of them the
    // cycle starts compacted (the rule of the compaction inside the cycle)
    std::vector<int32_t> live;
    for (int64_t j = 0; j < s; ++j) {
        bool lv = false;
        for (int cl = 0; cl < sh.n_clouds && !lv; ++cl) lv = act[(size_t)cl * s + j] != 0;
        if (lv) live.push_back((int32_t)j);
    }
    if (compact && !live.empty() && (int64_t)live.size() <= spmm_tile_width(s) / 2) {
        const int64_t s_new = (int64_t)live.size();
        CHAFF_HIP(hipMemcpyAsync(L.keep, live.data(), s_new * sizeof(int32_t), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL((k_start_vector_cols<C>), dim3(blocks_for(rows * s_new)), dim3(256), 0, st,
                           (const c128*)L.r, (const int32_t*)c->wire_cloud, (const double*)L.inv_rn, rows, s,
                           (const int32_t*)L.keep, s_new, r);
        CHAFF_LAUNCH_CHECK();
        if (!lazy) {
            const int64_t words = rows * s_new * (int64_t)sizeof(C) / 4;
            hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(words)), dim3(256), 0, st, (uint32_t*)xc, words);
            CHAFF_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(words)), dim3(256), 0, st, (uint32_t*)p, words);
            CHAFF_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(words)), dim3(256), 0, st, (uint32_t*)q, words);
            CHAFF_LAUNCH_CHECK();
        }
        chaff_status cst = cocg_narrow_shape(c, cs, Lc, L, colmap, live, st);
        if (cst != CHAFF_OK) return cst;
        if (g_verbose)
            std::fprintf(stderr, "[chaff] cocg cycle starts on %lld columns\n", (long long)cs.s);
    } else {
        hipLaunchKernelGGL((k_start_vector<C>), dim3(blocks_for(vs)), dim3(256), 0, st, (const c128*)L.r,
                           (const int32_t*)c->wire_cloud, (const double*)L.inv_rn, sh.n_clouds, rows, s, r);
        CHAFF_LAUNCH_CHECK();
        const int64_t words = vs * (int64_t)sizeof(C) / 4;
        if (!lazy) {
            hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(words)), dim3(256), 0, st, (uint32_t*)xc, words);
            CHAFF_LAUNCH_CHECK();
        }
        if ((first || !use_rr) && !lazy) {   // p and q enter the first step multiplied by zero: they must be finite
            hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(2 * words)), dim3(256), 0, st, (uint32_t*)p, 2 * words);
            CHAFF_LAUNCH_CHECK();
        }
    }
    CHAFF_HIP(hipStreamSynchronize(st));   // host staging vectors may leave scope
    int mode = (first || !use_rr) ? 0 : 2;
    int32_t last_checked = -1;
    bool pending_applied = false;   // set by a compaction, which applies the deferred x update itself
    std::vector<int32_t> flags;
    for (int k = 0; k <= o->restart; ++k) {
        const int wst = spmm_tile_width(cs.s);
        const bool first_step = lazy && k == 0;   // alpha = 0 and q holds nothing yet
        if (nbhd) {   // r -= alpha q, ||r||^2; then z = M r (over q) with per-tile r^T z
            {
                ProfScope pu(wst == 64 ? "k_cg_rupd" : "k_cg_rupd_narrow", st,
                             ((first_step ? 1.0 : 3.0) * rows * cs.s) * sizeof(C));
                switch (wst) {
                    case 1: launch_cg_rupd<C, 1>(cs, Lc, q, r, first_step, st); break;
                    case 2: launch_cg_rupd<C, 2>(cs, Lc, q, r, first_step, st); break;
                    case 4: launch_cg_rupd<C, 4>(cs, Lc, q, r, first_step, st); break;
                    case 8: launch_cg_rupd<C, 8>(cs, Lc, q, r, first_step, st); break;
                    case 16: launch_cg_rupd<C, 16>(cs, Lc, q, r, first_step, st); break;
                    case 32: launch_cg_rupd<C, 32>(cs, Lc, q, r, first_step, st); break;
                    default: launch_cg_rupd<C, 64>(cs, Lc, q, r, first_step, st); break;
                }
            }
            CHAFF_LAUNCH_CHECK();
            {
                ProfScope pm(cs.cocg_st == 64 ? "nbhd_apply" : "nbhd_apply_narrow", st,
                             ProfWork{((double)sizeof(CZ) * NB2 + 4.0) * c->nnzb + 4.0 * (c->n + 1) +
                                          2.0 * rows * cs.s * sizeof(C),
                                      8.0 * NB2 * (double)c->nnzb * cs.s});
                switch (cs.cocg_st) {
                    case 8: launch_cocg_spmm<CZ, C, 8>(c, cs, Lc, Pinv, r, q, st); break;
                    case 16: launch_cocg_spmm<CZ, C, 16>(c, cs, Lc, Pinv, r, q, st); break;
                    case 32: launch_cocg_spmm<CZ, C, 32>(c, cs, Lc, Pinv, r, q, st); break;
                    default: launch_cocg_spmm<CZ, C, 64>(c, cs, Lc, Pinv, r, q, st); break;
                }
            }
            CHAFF_LAUNCH_CHECK();
            group_sum(L.tpart, cs.s, 0, 0, 1, Lc.group_tile_off, cs.n_groups, cs.s, L.gpart, st);
            CHAFF_LAUNCH_CHECK();
            group_sum(L.gpart, cs.s, 0, 0, 1, Lc.cloud_group_off, cs.n_clouds, cs.s, L.h1, st);   // r^T z
            CHAFF_LAUNCH_CHECK();
            chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, cs.n_clouds, cs.nslot, 1, 1, cs.s,
                      L.h1 + cs.nsys, st);   // ||r||^2
        } else if (clus) {   // r -= alpha q, z = M r (over q), r^T z, ||r||^2
            ProfScope pu(wst == 64 ? "k_cg_update" : "k_cg_update_narrow", st,
                         ProfWork{(4.0 * rows * cs.s) * sizeof(C) + (double)cluster_count(c) * CLR2 * sizeof(CZ),
                                  8.0 * CLR2 * (double)cluster_count(c) * cs.s});
            switch (wst) {
                case 1: launch_cg_update_cl<CZ, C, 1>(cs, Lc, Mb, q, r, st); break;
                case 2: launch_cg_update_cl<CZ, C, 2>(cs, Lc, Mb, q, r, st); break;
                case 4: launch_cg_update_cl<CZ, C, 4>(cs, Lc, Mb, q, r, st); break;
                case 8: launch_cg_update_cl<CZ, C, 8>(cs, Lc, Mb, q, r, st); break;
                case 16: launch_cg_update_cl<CZ, C, 16>(cs, Lc, Mb, q, r, st); break;
                case 32: launch_cg_update_cl<CZ, C, 32>(cs, Lc, Mb, q, r, st); break;
                default: launch_cg_update_cl<CZ, C, 64>(cs, Lc, Mb, q, r, st); break;
            }
        } else {   // r -= alpha q, r^T (P r), ||r||^2 (alpha = 0 on entry)
            ProfScope pu(wst == 64 ? "k_cg_update" : "k_cg_update_narrow", st,
                         (3.0 * rows * cs.s) * sizeof(C) + (double)sh.n * NB2 * sizeof(CZ));
            const C* qc = q;
            switch (wst) {
                case 1: launch_cg_update<CZ, C, 1>(cs, Lc, Pinv, qc, r, st); break;
                case 2: launch_cg_update<CZ, C, 2>(cs, Lc, Pinv, qc, r, st); break;
                case 4: launch_cg_update<CZ, C, 4>(cs, Lc, Pinv, qc, r, st); break;
                case 8: launch_cg_update<CZ, C, 8>(cs, Lc, Pinv, qc, r, st); break;
                case 16: launch_cg_update<CZ, C, 16>(cs, Lc, Pinv, qc, r, st); break;
                case 32: launch_cg_update<CZ, C, 32>(cs, Lc, Pinv, qc, r, st); break;
                default: launch_cg_update<CZ, C, 64>(cs, Lc, Pinv, qc, r, st); break;
            }
        }
        CHAFF_LAUNCH_CHECK();
        if (!nbhd)
            chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, cs.n_clouds, cs.nslot, 0, 2, cs.s,
                      L.h1, st);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, st, (uint32_t*)L.counter, (int64_t)1);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cg_step, dim3(blocks_for(cs.nsys, 64)), dim3(64), 0, st, cs.nsys, (const c128*)L.h1,
                           (const c128*)(L.h1 + cs.nsys), mode, L.cg, L.counter, L.active);
        CHAFF_LAUNCH_CHECK();
        int32_t n_act = 0;
        CHAFF_HIP(hipMemcpyAsync(&n_act, L.counter, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CHAFF_HIP(hipStreamSynchronize(st));
        if (g_verbose && k % 50 == 0)
            std::fprintf(stderr, "[chaff] cocg step %d: %d of %lld systems above their checkpoint (%lld columns)\n",
                         k, n_act, (long long)cs.nsys, (long long)cs.s);
        if (n_act == 0) break;
        if (k == o->restart) {   // the step cap with systems still above their checkpoint
            capped = true;
            break;
        }
        if (compact && cs.s > 1 && n_act != last_checked && n_act <= (int64_t)cs.n_clouds * (wst / 2)) {
            last_checked = n_act;
            flags.resize(cs.nsys);
            CHAFF_HIP(hipMemcpyAsync(flags.data(), L.active, cs.nsys * sizeof(int32_t), hipMemcpyDeviceToHost, st));
            CHAFF_HIP(hipStreamSynchronize(st));
            std::vector<int32_t> keep;
            for (int64_t j = 0; j < cs.s; ++j) {
                bool live = false;
                for (int cl = 0; cl < cs.n_clouds && !live; ++cl) live = flags[(int64_t)cl * cs.s + j] != 0;
                if (live) keep.push_back((int32_t)j);
            }
            if (!keep.empty() && (int64_t)keep.size() <= wst / 2) {
                chaff_status cst =
                    cocg_compact<C>(c, cs, Lc, L, colmap, keep, s, xc, r, p, q, zq, xc_valid, p_valid, st);
                if (cst != CHAFF_OK) return cst;
                pending_applied = true;
                xc_valid = true;   // the compaction clears the new x_c
                if (g_verbose)
                    std::fprintf(stderr, "[chaff] cocg step %d: compacted to %lld columns\n", k, (long long)cs.s);
            }
        }
        mode = 1;
        ++iters;
        if (zq) {   // x += alpha p_old (deferred), p = z + beta p_old
            const bool pfirst = !p_valid;   // the first direction: p = z, nothing to add to x
            const int pend = (pending_applied || pfirst) ? 0 : (xc_valid ? 1 : 2);
            pending_applied = false;
            p_valid = true;
            if (pend == 2) xc_valid = true;
            ProfScope pp(spmm_tile_width(cs.s) == 64 ? "k_cg_p" : "k_cg_p_narrow", st,
                         (pfirst ? 2.0 : 3.0 + (pend == 2 ? 1.0 : 2.0 * pend)) * rows * cs.s * sizeof(C));
            const C* zc = q;
            switch (spmm_tile_width(cs.s)) {
                case 1: launch_cg_pdir_z<C, 1>(cs, Lc, zc, p, xc, pend, pfirst, st); break;
                case 2: launch_cg_pdir_z<C, 2>(cs, Lc, zc, p, xc, pend, pfirst, st); break;
                case 4: launch_cg_pdir_z<C, 4>(cs, Lc, zc, p, xc, pend, pfirst, st); break;
                case 8: launch_cg_pdir_z<C, 8>(cs, Lc, zc, p, xc, pend, pfirst, st); break;
                case 16: launch_cg_pdir_z<C, 16>(cs, Lc, zc, p, xc, pend, pfirst, st); break;
                case 32: launch_cg_pdir_z<C, 32>(cs, Lc, zc, p, xc, pend, pfirst, st); break;
                default: launch_cg_pdir_z<C, 64>(cs, Lc, zc, p, xc, pend, pfirst, st); break;
            }
        } else {   // x += alpha p_old (deferred), p = P r + beta p_old
            const int pend = pending_applied ? 0 : 1;
            pending_applied = false;
            ProfScope pp(spmm_tile_width(cs.s) == 64 ? "k_cg_p" : "k_cg_p_narrow", st,
                         (3.0 + 2.0 * pend) * rows * cs.s * sizeof(C) + (double)sh.n * NB2 * sizeof(CZ));
            const int ws2 = spmm_tile_width(cs.s);
            const C* rc_ = r;
            switch (ws2) {
                case 1: launch_cg_pdir<CZ, C, 1>(cs, Lc, Pinv, rc_, p, xc, pend, st); break;
                case 2: launch_cg_pdir<CZ, C, 2>(cs, Lc, Pinv, rc_, p, xc, pend, st); break;
                case 4: launch_cg_pdir<CZ, C, 4>(cs, Lc, Pinv, rc_, p, xc, pend, st); break;
                case 8: launch_cg_pdir<CZ, C, 8>(cs, Lc, Pinv, rc_, p, xc, pend, st); break;
                case 16: launch_cg_pdir<CZ, C, 16>(cs, Lc, Pinv, rc_, p, xc, pend, st); break;
                case 32: launch_cg_pdir<CZ, C, 32>(cs, Lc, Pinv, rc_, p, xc, pend, st); break;
                default: launch_cg_pdir<CZ, C, 64>(cs, Lc, Pinv, rc_, p, xc, pend, st); break;
            }
        }
        CHAFF_LAUNCH_CHECK();
        {   // q = Z p with per-tile p^T q
            // full-width launches are timed apart from the narrower ones after a compaction
            // algorithmic work: Z with its column indices and row pointers once,
            // p gathered once and q written once; 8 NB^2 flops per block and column
            ProfScope ps(cs.cocg_st == 64 ? "spmm" : "spmm_narrow", st,
                         ProfWork{((double)sizeof(CZ) * NB2 + 4.0) * c->nnzb + 4.0 * (c->n + 1) +
                                      2.0 * rows * cs.s * sizeof(C),
                                  8.0 * NB2 * (double)c->nnzb * cs.s});
            switch (cs.cocg_st) {
                case 8: launch_cocg_spmm<CZ, C, 8>(c, cs, Lc, Z, p, q, st); break;
                case 16: launch_cocg_spmm<CZ, C, 16>(c, cs, Lc, Z, p, q, st); break;
                case 32: launch_cocg_spmm<CZ, C, 32>(c, cs, Lc, Z, p, q, st); break;
                default: launch_cocg_spmm<CZ, C, 64>(c, cs, Lc, Z, p, q, st); break;
            }
        }
        CHAFF_LAUNCH_CHECK();
        // sigma: tiles -> groups -> clouds, fixed order
        group_sum(L.tpart, cs.s, 0, 0, 1, Lc.group_tile_off, cs.n_groups, cs.s, L.gpart, st);
        CHAFF_LAUNCH_CHECK();
        group_sum(L.gpart, cs.s, 0, 0, 1, Lc.cloud_group_off, cs.n_clouds, cs.s, L.nrm, st);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cg_alpha, dim3(blocks_for(cs.nsys, 64)), dim3(64), 0, st, cs.nsys, (const c128*)L.nrm,
                           L.cg);
        CHAFF_LAUNCH_CHECK();
    }
    // the deferred x update of the last step, then x64 += scale * xc (one pass)
    if (p_valid) {
        hipLaunchKernelGGL((k_cg_flush<C>), dim3(blocks_for(rows * cs.s)), dim3(256), 0, st,
                           (const int32_t*)c->wire_cloud, (const CgState*)L.cg, (const double*)L.rn,
                           (const int32_t*)L.colmap, rows, cs.s, s, (const C*)p,
                           xc_valid ? (const C*)xc : (const C*)nullptr, L.x);
        CHAFF_LAUNCH_CHECK();
    }
    return CHAFF_OK;
}

// ------------------------------------------------------------------ GCR (Sec. II-B)

// 1 / ||Q_j|| per system; a finished system gets 0, and a vanishing Q_j (no
// new direction) finishes the system for the rest of the cycle
__global__ void k_gcr_beta(int64_t nsys, const c128* __restrict__ nrm2, SysState* __restrict__ sys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsys) return;
    SysState S = sys[i];
    const double b2 = nrm2[i].re;
    if (!S.done && !(b2 > 1e-300 && isfinite(b2))) S.done = 1;
    S.inv_beta = S.done ? 0.0 : 1.0 / sqrt(b2);
    sys[i] = S;
}

// Q_j *= inv_beta, U_j *= inv_beta (per system)
template <typename C>
__global__ void k_gcr_scale(C* __restrict__ Q, C* __restrict__ U, const int32_t* __restrict__ wire_cloud,
                            const SysState* __restrict__ sys, int64_t n_rows, int64_t s) {
    using R = typename real_of<C>::type;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s) return;
    const int64_t row = t / s, r = t - (t / s) * s;
    const R f = (R)sys[(int64_t)wire_cloud[row / NB] * s + r].inv_beta;
    Q[t] = cscale(Q[t], f);
    U[t] = cscale(U[t], f);
}

// alpha = Q_j^H rho (0 for finished systems), and -alpha
__global__ void k_gcr_alpha(int64_t nsys, const c128* __restrict__ dot, const SysState* __restrict__ sys,
                            c128* __restrict__ alpha, c128* __restrict__ neg_alpha) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsys) return;
    const c128 a = sys[i].done ? c128{0, 0} : dot[i];
    alpha[i] = a;
    neg_alpha[i] = c128{-a.re, -a.im};
}

// ||rho|| (relative to the cycle start) against the system's target; counts
// the systems still running
__global__ void k_gcr_check(int64_t nsys, const c128* __restrict__ nrm2, SysState* __restrict__ sys,
                            int32_t* __restrict__ n_active) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsys) return;
    SysState S = sys[i];
    if (S.done) return;
    S.est = sqrt(fmax(nrm2[i].re, 0.0));
    if (S.est <= S.target || !isfinite(S.est)) S.done = 1;
    else atomicAdd(n_active, 1);
    sys[i] = S;
}

// x += ||r|| xc (FP64 solution, per system)
template <typename C>
__global__ void k_gcr_finish(const C* __restrict__ xc, const int32_t* __restrict__ wire_cloud,
                             const double* __restrict__ rn, int64_t n_rows, int64_t s, c128* __restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rows * s) return;
    const int64_t row = t / s, r = t - (t / s) * s;
    const double f = rn[(int64_t)wire_cloud[row / NB] * s + r];
    const c128 v = ccast<c128>(xc[t]);
    x[t] = c128{x[t].re + f * v.re, x[t].im + f * v.im};
}

// One restarted GCR(m) cycle, right-preconditioned, every system in lockstep
// with its own coefficients.  rho = r / ||r|| is the working residual and xc
// the correction (precision C).  Step j: U_j = P rho and Q_j = Z U_j; two
// classical Gram-Schmidt passes make Q_j orthogonal (Hermitian products) to
// Q_0 .. Q_{j-1}, the same combinations are applied to U_j so that Q_j = Z U_j
// keeps holding, and both are scaled to ||Q_j|| = 1; then alpha = Q_j^H rho,
// rho -= alpha Q_j (minimal residual over the directions so far) and
// xc += alpha U_j.  A system stops once ||rho|| reaches its target; at the end
// x += ||r|| xc.  L.sys, L.rn and L.inv_rn are set by the caller.
template <typename C, typename CZ>
static chaff_status gcr_cycle(Cloud* c, const chaff_solve_opts* o, const SolveShape& sh, SolveLayout& L,
                              const CZ* Z, const CZ* Pinv, int& iters, hipStream_t st) {
    const int64_t rows = sh.rows, s = sh.s, vs = rows * s, nsys = sh.nsys;
    const int m = sh.m;
    C* V = static_cast<C*>(L.V);
    C* U = V;                                  // U_j = V[j]
    C* Q = V + (int64_t)m * vs;                // Q_j = V[m + j]
    C* rho = V + (int64_t)2 * m * vs;
    C* xc = rho + vs;
    const int wst = spmm_tile_width(s);
    const dim3 grid(sh.n_chunks, (unsigned)((s + wst - 1) / wst));
    const int32_t* wc = (const int32_t*)c->wire_cloud;
    const int norm_slot = sh.nslot - 1;
    hipLaunchKernelGGL((k_start_vector<C>), dim3(blocks_for(vs)), dim3(256), 0, st, (const c128*)L.r, wc,
                       (const double*)L.inv_rn, sh.n_clouds, rows, s, rho);
    CHAFF_LAUNCH_CHECK();
    const int64_t xc_words = vs * (int64_t)(sizeof(C) / 4);
    hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(xc_words, 256)), dim3(256), 0, st, (uint32_t*)xc, xc_words);
    CHAFF_LAUNCH_CHECK();
    chaff_status sst;
    for (int j = 0; j < m; ++j) {
        ++iters;
        C* uj = U + (int64_t)j * vs;
        C* qj = Q + (int64_t)j * vs;
        if (o->precond == CHAFF_PRECOND_CLUSTER)
            sst = cluster_apply_launch(c, (chaff_prec)o->prec, Pinv, rho, sizeof(C) == 16, uj, sizeof(C) == 16,
                                       false, s, st, "precond");
        else if (o->precond == CHAFF_PRECOND_NBHD)
            sst = spmm_launch<CZ, C, C, 0, false>(c->row_ptr, c->col_idx, Pinv, rho, (const C*)nullptr, uj, c->n,
                                                  c->nnzb, s, o->spmm_variant, st, "precond");
        else
            sst = spmm_launch<CZ, C, C, 0, true>(nullptr, nullptr, Pinv, rho, (const C*)nullptr, uj, c->n, c->n, s,
                                                 -1, st, "precond");
        if (sst != CHAFF_OK) return sst;
        sst = spmm_launch<CZ, C, C, 0, false>(c->row_ptr, c->col_idx, Z, uj, (const C*)nullptr, qj, c->n, c->nnzb,
                                              s, o->spmm_variant, st);
        if (sst != CHAFF_OK) return sst;
        for (int pass = 0; pass < 2 && j > 0; ++pass) {   // classical Gram-Schmidt, twice
            for (int i0 = 0; i0 < j; i0 += GV) {
                ProfScope p1("k_dots", st, (double)(std::min(GV, j - i0) + 1) * vs * sizeof(C));
                hipLaunchKernelGGL((k_dots<C>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)Q, vs, i0,
                                   std::min(GV, j - i0), (const C*)qj, s, wst, L.part, sh.nslot);
                CHAFF_LAUNCH_CHECK();
            }
            chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, 0, j, s,
                      L.h1, st);
            CHAFF_LAUNCH_CHECK();
            ProfScope p2("k_update", st, (double)(2 * j + 4) * vs * sizeof(C));
            hipLaunchKernelGGL((k_update<C, false>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)Q, vs,
                               j, (const c128*)L.h1, sh.n_clouds, qj, s, wst, L.part, sh.nslot, 0);
            CHAFF_LAUNCH_CHECK();
            hipLaunchKernelGGL((k_update<C, false>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)U, vs,
                               j, (const c128*)L.h1, sh.n_clouds, uj, s, wst, L.part, sh.nslot, 0);
            CHAFF_LAUNCH_CHECK();
        }
        hipLaunchKernelGGL((k_norm2<C>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)qj, s, wst, L.part,
                           sh.nslot, norm_slot);
        CHAFF_LAUNCH_CHECK();
        chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, norm_slot, 1, s,
                  L.nrm, st);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gcr_beta, dim3(blocks_for(nsys, 64)), dim3(64), 0, st, nsys, (const c128*)L.nrm, L.sys);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_gcr_scale<C>), dim3(blocks_for(vs)), dim3(256), 0, st, qj, uj, wc,
                           (const SysState*)L.sys, rows, s);
        CHAFF_LAUNCH_CHECK();
        // alpha = Q_j^H rho; rho -= alpha Q_j (with ||rho||^2); xc += alpha U_j
        hipLaunchKernelGGL((k_dots<C>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)qj, vs, 0, 1,
                           (const C*)rho, s, wst, L.part, sh.nslot);
        CHAFF_LAUNCH_CHECK();
        chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, 0, 1, s, L.h2, st);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gcr_alpha, dim3(blocks_for(nsys, 64)), dim3(64), 0, st, nsys, (const c128*)L.h2,
                           (const SysState*)L.sys, L.Y, L.G);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_update<C, true>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)qj, vs, 1,
                           (const c128*)L.Y, sh.n_clouds, rho, s, wst, L.part, sh.nslot, norm_slot);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_update<C, false>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)uj, vs, 1,
                           (const c128*)L.G, sh.n_clouds, xc, s, wst, L.part, sh.nslot, 0);
        CHAFF_LAUNCH_CHECK();
        chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, norm_slot, 1, s,
                  L.nrm, st);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, st, (uint32_t*)L.counter, (int64_t)1);
        hipLaunchKernelGGL(k_gcr_check, dim3(blocks_for(nsys, 64)), dim3(64), 0, st, nsys, (const c128*)L.nrm, L.sys,
                           L.counter);
        CHAFF_LAUNCH_CHECK();
        int32_t n_act = 0;
        CHAFF_HIP(hipMemcpyAsync(&n_act, L.counter, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CHAFF_HIP(hipStreamSynchronize(st));
        if (n_act == 0) break;
    }
    hipLaunchKernelGGL((k_gcr_finish<C>), dim3(blocks_for(vs)), dim3(256), 0, st, (const C*)xc, wc,
                       (const double*)L.rn, rows, s, L.x);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

template <typename C, typename CZ>
static chaff_status solve_impl(Cloud* c, const chaff_solve_opts* o, const CZ* Z, const CZ* Pinv,
                               const double* k_hat, const double* e_hat, int64_t s, c128* Xout, void* ws,
                               size_t ws_bytes, chaff_solve_stats* stats, double* rel_res_out, hipStream_t st) {
    auto t_start = std::chrono::steady_clock::now();
    const int m = o->restart;
    SolveShape sh = solve_shape(c, m, s, (chaff_prec)o->prec, o->method);
    SolveLayout L = carve_solve(ws, ws_bytes, sh);
    if (L.bytes > ws_bytes)
        return fail(CHAFF_EWORKSPACE, "solve workspace too small: need " + std::to_string(L.bytes));
    if (o->precond == CHAFF_PRECOND_CLUSTER && NB != 7)
        return fail(CHAFF_EINVAL, "the cluster preconditioner needs wires of 8 segments");
    if (o->precond == CHAFF_PRECOND_CLUSTER) {
        chaff_status ck = cluster_check_table(c, Pinv, st);
        if (ck != CHAFF_OK) return ck;
    }
    if (o->precond == CHAFF_PRECOND_NBHD) {   // from here on Pinv points at M's blocks (Z's pattern)
        if (NB != 7) return fail(CHAFF_EINVAL, "the neighbourhood-inverse preconditioner needs wires of 8 segments");
        int size = 0;
        chaff_status ck = nbhd_check(c, (chaff_prec)o->prec, Pinv, &size, st);
        if (ck != CHAFF_OK) return ck;
        Pinv = reinterpret_cast<const CZ*>(reinterpret_cast<const char*>(Pinv) + nbhd_blocks_offset(c->n, size));
    }
    const int64_t rows = sh.rows, vs = rows * s, nsys = sh.nsys;
    C* V = static_cast<C*>(L.V);
    C* W = static_cast<C*>(L.W);
    C* T = static_cast<C*>(L.T);
    const int wst = spmm_tile_width(s);
    const unsigned ry = (unsigned)((s + wst - 1) / wst);

    // --- chunk tables (host -> device)
    {
        const int64_t cw = chunk_wires(c->n, o->method);
        std::vector<Chunk> ch;
        std::vector<int32_t> off(sh.n_clouds + 1, 0);
        int64_t cl_base = 0;   // clusters of the clouds before k
        for (int k = 0; k < sh.n_clouds; ++k) {
            off[k] = (int32_t)ch.size();
            for (int64_t w0 = c->cloud_off[k]; w0 < c->cloud_off[k + 1]; w0 += cw)
                ch.push_back(Chunk{w0, std::min<int64_t>(w0 + cw, c->cloud_off[k + 1]), k,
                                   (int32_t)(cl_base + (w0 - c->cloud_off[k]) / CLW)});
            cl_base += (c->cloud_off[k + 1] - c->cloud_off[k] + CLW - 1) / CLW;
        }
        off[sh.n_clouds] = (int32_t)ch.size();
        if (!ch.empty())
            CHAFF_HIP(hipMemcpyAsync(L.chunks, ch.data(), ch.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
        CHAFF_HIP(hipMemcpyAsync(L.cloud_chunk_off, off.data(), off.size() * sizeof(int32_t),
                                 hipMemcpyHostToDevice, st));
        // COCG product tiles (cloud-aligned) and their groups (cloud-aligned)
        std::vector<Chunk> tl;
        std::vector<int32_t> gto, cgo(sh.n_clouds + 1, 0);
        if (sh.method == CHAFF_COCG || sh.method == CHAFF_COCG_RR) {
            build_tiles(c, sh.tile_w, tl, gto, cgo);
            if (!tl.empty())
                CHAFF_HIP(hipMemcpyAsync(L.tiles, tl.data(), tl.size() * sizeof(Chunk), hipMemcpyHostToDevice, st));
            CHAFF_HIP(hipMemcpyAsync(L.group_tile_off, gto.data(), gto.size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice, st));
            CHAFF_HIP(hipMemcpyAsync(L.cloud_group_off, cgo.data(), cgo.size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice, st));
        }
        CHAFF_HIP(hipStreamSynchronize(st));  // host vectors go out of scope
    }

    // --- excitation and initial guess (internal order, FP64)
    chaff_status sst0 = CHAFF_OK;
    const double k = 2.0 * PI_K / c->wavelength;
    // complex64 with the neighbourhood inverse: the guess x0 = M u is formed in
    // FP32 from an FP32 copy of u (a guess needs no more), and x0's FP32 values,
    // widened exactly into the FP64 solution, give the first residual through
    // FP32 slabs (half the gathered bytes of FP64 ones) with FP64 accumulation
    const bool guess32 = std::is_same<C, c64>::value && o->use_x0 == 2 && o->precond == CHAFF_PRECOND_NBHD;
    c64* const u32 = guess32 ? reinterpret_cast<c64*>(V + vs) : nullptr;   // idle Krylov vectors
    c64* const x32 = guess32 ? reinterpret_cast<c64*>(V) : nullptr;
    hipLaunchKernelGGL(k_excitation, dim3(blocks_for(c->n * s)), dim3(256), 0, st, (const Wire*)c->wires,
                       (const int32_t*)nullptr, c->n, k_hat, e_hat, s, k, L.b, u32);
    CHAFF_LAUNCH_CHECK();
    if (guess32) {
        sst0 = spmm_launch<CZ, c64, c64, 0, false>(c->row_ptr, c->col_idx, Pinv, (const c64*)u32, (const c64*)nullptr,
                                                   x32, c->n, c->nnzb, s, -1, st, "guess_nbhd");
        if (sst0 != CHAFF_OK) return sst0;
        hipLaunchKernelGGL(k_widen, dim3(blocks_for(vs)), dim3(256), 0, st, (const c64*)x32, vs, L.x);
    } else if (o->use_x0 == 1) {
        hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for(vs)), dim3(256), 0, st, (const c128*)Xout,
                           (const int32_t*)c->perm, c->n, s, L.x, 0);
    } else if (o->use_x0 == 2 && o->precond == CHAFF_PRECOND_NBHD) {
        // neighbourhood-inverse guess x0 = M u (FP64 vectors, stored blocks on Z's pattern)
        sst0 = spmm_launch<CZ, c128, c128, 0, false>(c->row_ptr, c->col_idx, Pinv, (const c128*)L.b,
                                                     (const c128*)nullptr, L.x, c->n, c->nnzb, s, -1, st,
                                                     "guess_nbhd");
        if (sst0 != CHAFF_OK) return sst0;
    } else if (o->use_x0 == 2 && o->precond == CHAFF_PRECOND_CLUSTER) {
        // cluster guess x0 = M u (FP64 vectors, stored blocks)
        sst0 = cluster_apply_launch(c, (chaff_prec)o->prec, Pinv, L.b, true, L.x, true, false, s, st,
                                    "guess_cluster");
        if (sst0 != CHAFF_OK) return sst0;
    } else if (o->use_x0 == 2) {
        // block-Jacobi guess x0 = Pinv u (FP64 vectors, stored Pinv)
        sst0 = spmm_launch<CZ, c128, c128, 0, true>(nullptr, nullptr, Pinv, (const c128*)L.b, (const c128*)nullptr,
                                                    L.x, c->n, c->n, s, -1, st, "guess_block_jacobi");
        if (sst0 != CHAFF_OK) return sst0;
    } else {
        hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(vs * 4, 256)), dim3(256), 0, st, (uint32_t*)L.x,
                           vs * 4);
    }
    CHAFF_LAUNCH_CHECK();
    chaff_status sst = norms_to<c128>(sh, L, L.b, L.red, st);
    if (sst != CHAFF_OK) return sst;
    std::vector<c128> hb(nsys), hr(nsys);
    CHAFF_HIP(hipMemcpyAsync(hb.data(), L.red, nsys * sizeof(c128), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipStreamSynchronize(st));
    std::vector<double> bnorm(nsys), rel(nsys, 0.0);
    for (int64_t i = 0; i < nsys; ++i) bnorm[i] = std::sqrt(std::max(hb[i].re, 0.0));

    const bool refine = std::is_same<C, c64>::value;
    int cycles = 0, iters = 0;
    bool converged = false, broken = false, rr_restart = false;
    std::vector<double> hinv(nsys), hrn(nsys), cocg_scale;
    std::vector<SysState> hsys(nsys);
    for (;;) {
        // true residual r = b - Z x (FP64 accumulation over the stored Z)
        if (cycles == 0 && o->use_x0 == 0) {
            hipLaunchKernelGGL(k_copy_c128, dim3(blocks_for(vs)), dim3(256), 0, st, (const c128*)L.b, vs, L.r);
            CHAFF_LAUNCH_CHECK();
        } else if (cycles == 0 && guess32) {   // x = x32 exactly: the FP32 slabs give the same residual
            sst = spmm_launch<CZ, c64, c128, 1, false>(c->row_ptr, c->col_idx, Z, (const c64*)x32, L.b, L.r, c->n,
                                                       c->nnzb, s, -1, st, "spmm_residual_fp64");
            if (sst != CHAFF_OK) return sst;
        } else {
            sst = spmm_launch<CZ, c128, c128, 1, false>(c->row_ptr, c->col_idx, Z, L.x, L.b, L.r, c->n, c->nnzb, s, -1, st,
                                                        "spmm_residual_fp64");
            if (sst != CHAFF_OK) return sst;
        }
        sst = norms_to<c128>(sh, L, L.r, L.red, st);
        if (sst != CHAFF_OK) return sst;
        CHAFF_HIP(hipMemcpyAsync(hr.data(), L.red, nsys * sizeof(c128), hipMemcpyDeviceToHost, st));
        CHAFF_HIP(hipStreamSynchronize(st));
        double worst = 0.0;
        int64_t active = 0;
        broken = false;
        for (int64_t i = 0; i < nsys; ++i) {
            double rn = std::sqrt(std::max(hr[i].re, 0.0));
            rel[i] = bnorm[i] > 0 ? rn / bnorm[i] : 0.0;
            if (!std::isfinite(hr[i].re)) {   // a recurrence broke down and left x non-finite
                rel[i] = INFINITY;
                broken = true;
            }
            worst = std::max(worst, rel[i]);
            bool act = rel[i] > o->tol && std::isfinite(rel[i]);
            active += act;
            hrn[i] = act ? rn : 0.0;
            hinv[i] = act ? 1.0 / rn : 0.0;
            SysState S{};
            S.done = act ? 0 : 1;
            S.k_used = 0;
            S.inv_beta = 0.0;
            S.est = 1.0;
            // FP32 cycles aim at a fixed reduction; FP64 cycles straight at the target
            double need = act ? (o->tol * bnorm[i] / rn) : 1.0;
            S.target = refine ? std::max(o->inner_tol, std::min(need, 1.0) * 0.5) : std::min(need * 0.5, 1.0);
            hsys[i] = S;
        }
        if (g_verbose)
            std::fprintf(stderr, "[chaff] cycle %d: active %lld max rel residual %.3e (iterations so far %d)\n",
                         cycles, (long long)active, worst, iters);
        if (active == 0) { converged = !broken; break; }
        if (cycles >= o->max_cycles) break;
        ++cycles;
        CHAFF_HIP(hipMemcpyAsync(L.rn, hrn.data(), nsys * sizeof(double), hipMemcpyHostToDevice, st));
        CHAFF_HIP(hipMemcpyAsync(L.inv_rn, hinv.data(), nsys * sizeof(double), hipMemcpyHostToDevice, st));
        if (sh.method == CHAFF_COCG || sh.method == CHAFF_COCG_RR) {
            // fixed per-system scale for the whole run (set by the first cycle)
            const bool first = cocg_scale.empty();
            if (first) cocg_scale.assign(nsys, 0.0);
            std::vector<double> tg(nsys), ck(nsys), sc_inv(nsys), sc(nsys);
            std::vector<int32_t> act(nsys);
            for (int64_t i = 0; i < nsys; ++i) {
                const double rn = std::sqrt(std::max(hr[i].re, 0.0));
                if (cocg_scale[i] <= 0.0) cocg_scale[i] = rn > 0 ? rn : 1.0;
                sc[i] = hsys[i].done ? 0.0 : cocg_scale[i];
                sc_inv[i] = hsys[i].done ? 0.0 : 1.0 / cocg_scale[i];
                act[i] = hsys[i].done ? 0 : 1;
                tg[i] = 0.5 * o->tol * bnorm[i] / cocg_scale[i];
                ck[i] = std::max(tg[i], o->inner_tol * rn / cocg_scale[i]);
            }
            CHAFF_HIP(hipMemcpyAsync(L.rn, sc.data(), nsys * sizeof(double), hipMemcpyHostToDevice, st));
            CHAFF_HIP(hipMemcpyAsync(L.inv_rn, sc_inv.data(), nsys * sizeof(double), hipMemcpyHostToDevice, st));
            // COCG_RR carries p and r^T z into the next cycle; after a cycle that
            // stalled at its step cap the recurrence restarts from the true residual
            // instead (a stagnating FP32 recurrence carried on can overflow)
            bool capped = false;
            sst = cocg_cycle<C, CZ>(c, o, sh, L, Z, Pinv, tg, ck, act, first || rr_restart, iters, capped, st);
            if (sst != CHAFF_OK) return sst;
            rr_restart = capped;
            continue;
        }
        CHAFF_HIP(hipMemcpyAsync(L.sys, hsys.data(), nsys * sizeof(SysState), hipMemcpyHostToDevice, st));
        if (sh.method == CHAFF_GCR) {
            sst = gcr_cycle<C, CZ>(c, o, sh, L, Z, Pinv, iters, st);
            if (sst != CHAFF_OK) return sst;
            continue;
        }
        // g = e_1 for every system
        {
            std::vector<c128> g0((size_t)nsys * (m + 1), c128{0, 0});
            for (int64_t i = 0; i < nsys; ++i) g0[(size_t)i * (m + 1)] = c128{1, 0};
            CHAFF_HIP(hipMemcpyAsync(L.G, g0.data(), g0.size() * sizeof(c128), hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL((k_start_vector<C>), dim3(blocks_for(vs)), dim3(256), 0, st, (const c128*)L.r,
                               (const int32_t*)c->wire_cloud, (const double*)L.inv_rn, sh.n_clouds, rows, s, V);
            CHAFF_LAUNCH_CHECK();
            CHAFF_HIP(hipStreamSynchronize(st));
        }
        int j = 0;
        for (; j < m; ++j) {
            ++iters;
            C* vj = V + (int64_t)j * vs;
            // W = Z P v_j
            if (o->precond == CHAFF_PRECOND_CLUSTER)
                sst = cluster_apply_launch(c, (chaff_prec)o->prec, Pinv, vj, sizeof(C) == 16, T, sizeof(C) == 16,
                                           false, s, st, "precond");
            else if (o->precond == CHAFF_PRECOND_NBHD)
                sst = spmm_launch<CZ, C, C, 0, false>(c->row_ptr, c->col_idx, Pinv, vj, (const C*)nullptr, T, c->n,
                                                      c->nnzb, s, o->spmm_variant, st, "precond");
            else
                sst = spmm_launch<CZ, C, C, 0, true>(nullptr, nullptr, Pinv, vj, (const C*)nullptr, T, c->n, c->n, s,
                                                     -1, st, "precond");
            if (sst != CHAFF_OK) return sst;
            sst = spmm_launch<CZ, C, C, 0, false>(c->row_ptr, c->col_idx, Z, T, (const C*)nullptr, W, c->n, c->nnzb,
                                                  s, o->spmm_variant, st);
            if (sst != CHAFF_OK) return sst;
            const int nv = j + 1;
            dim3 grid(sh.n_chunks, ry);
            {  // classical Gram-Schmidt, twice, and the new vector's norm
            // CGS pass 1
            for (int i0 = 0; i0 < nv; i0 += GV) {
                ProfScope p1("k_dots", st, (double)(std::min(GV, nv - i0) + 1) * vs * sizeof(C));
                hipLaunchKernelGGL((k_dots<C>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)V, vs, i0,
                                   std::min(GV, nv - i0), (const C*)W, s, wst, L.part, sh.nslot);
                CHAFF_LAUNCH_CHECK();
            }
            chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, 0, nv,
                               s, L.h1, st);
            CHAFF_LAUNCH_CHECK();
            {
                ProfScope p2("k_update", st, (double)(nv + 2) * vs * sizeof(C));
                hipLaunchKernelGGL((k_update<C, false>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)V,
                                   vs, nv, (const c128*)L.h1, sh.n_clouds, W, s, wst, L.part, sh.nslot, 0);
            }
            CHAFF_LAUNCH_CHECK();
            // CGS pass 2 (re-orthogonalisation) + norm
            for (int i0 = 0; i0 < nv; i0 += GV) {
                ProfScope p1("k_dots", st, (double)(std::min(GV, nv - i0) + 1) * vs * sizeof(C));
                hipLaunchKernelGGL((k_dots<C>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)V, vs, i0,
                                   std::min(GV, nv - i0), (const C*)W, s, wst, L.part, sh.nslot);
                CHAFF_LAUNCH_CHECK();
            }
            chunk_sum((const c128*)L.part, (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, 0, nv,
                               s, L.h2, st);
            CHAFF_LAUNCH_CHECK();
            {
                ProfScope p3("k_update_norm", st, (double)(nv + 2) * vs * sizeof(C));
                hipLaunchKernelGGL((k_update<C, true>), grid, dim3(RB), 0, st, (const Chunk*)L.chunks, (const C*)V,
                                   vs, nv, (const c128*)L.h2, sh.n_clouds, W, s, wst, L.part, sh.nslot,
                                   sh.nslot - 1);
            }
            CHAFF_LAUNCH_CHECK();
            chunk_sum((const c128*)L.part,
                               (const int32_t*)L.cloud_chunk_off, sh.n_clouds, sh.nslot, sh.nslot - 1, 1, s, L.nrm, st);
            CHAFF_LAUNCH_CHECK();
            }
            hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(64), 0, st, (uint32_t*)L.counter, (int64_t)1);
            CHAFF_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_givens, dim3(blocks_for(nsys, 64)), dim3(64), 0, st, nsys, j, m, (const c128*)L.h1,
                               (const c128*)L.h2, (const c128*)L.nrm, L.H, L.G, L.cs, L.sn, L.sys, L.counter);
            CHAFF_LAUNCH_CHECK();
            if (j + 1 < m) {
                hipLaunchKernelGGL((k_scale_next<C>), dim3(blocks_for(vs)), dim3(256), 0, st, (const C*)W,
                                   (const int32_t*)c->wire_cloud, (const SysState*)L.sys, rows, s,
                                   V + (int64_t)(j + 1) * vs);
                CHAFF_LAUNCH_CHECK();
            }
            int32_t n_act = 0;
            CHAFF_HIP(hipMemcpyAsync(&n_act, L.counter, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            CHAFF_HIP(hipStreamSynchronize(st));
            if (n_act == 0) break;
        }
        // x += P (V y)
        const int nv_max = std::min(j + 1, m);
        hipLaunchKernelGGL(k_lsq, dim3(blocks_for(nsys, 64)), dim3(64), 0, st, nsys, m, (const c128*)L.H,
                           (const c128*)L.G, (const SysState*)L.sys, (const double*)L.rn, L.Y, nv_max);
        CHAFF_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_combine<C>), dim3(blocks_for(vs)), dim3(256), 0, st, (const C*)V, vs, nv_max,
                           (const c128*)L.Y, (const int32_t*)c->wire_cloud, sh.n_clouds, rows, s, T);
        CHAFF_LAUNCH_CHECK();
        if (o->precond == CHAFF_PRECOND_CLUSTER)
            sst = cluster_apply_launch(c, (chaff_prec)o->prec, Pinv, T, sizeof(C) == 16, L.x, true, true, s, st,
                                       "precond_update_fp64");
        else if (o->precond == CHAFF_PRECOND_NBHD)
            sst = spmm_launch<CZ, C, c128, 2, false>(c->row_ptr, c->col_idx, Pinv, T, (const c128*)nullptr, L.x,
                                                     c->n, c->nnzb, s, -1, st, "precond_update_fp64");
        else
            sst = spmm_launch<CZ, C, c128, 2, true>(nullptr, nullptr, Pinv, T, (const c128*)nullptr, L.x, c->n, c->n,
                                                    s, -1, st, "precond_update_fp64");
        if (sst != CHAFF_OK) return sst;
    }
    // --- output (caller order)
    hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for(vs)), dim3(256), 0, st, (const c128*)L.x,
                       (const int32_t*)c->perm, c->n, s, Xout, 1);
    CHAFF_LAUNCH_CHECK();
    CHAFF_HIP(hipStreamSynchronize(st));
    double worst = 0.0;
    for (int64_t i = 0; i < nsys; ++i) worst = std::max(worst, rel[i]);
    if (rel_res_out)
        for (int64_t i = 0; i < nsys; ++i) rel_res_out[i] = rel[i];
    if (stats) {
        stats->cycles = cycles;
        stats->iterations = iters;
        stats->max_rel_residual = worst;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (!converged)
        return fail(CHAFF_ENOCONV, (broken ? "breakdown (non-finite solution) after " : "no convergence after ") +
                                       std::to_string(cycles) + " cycles; max relative residual " +
                                       std::to_string(worst));
    return CHAFF_OK;
}

chaff_status solve(Cloud* c, const chaff_solve_opts* o, const void* Z, const void* Pinv, const double* k_hat,
                   const double* e_hat, int64_t s, void* X, void* ws, size_t ws_bytes, chaff_solve_stats* st_out,
                   double* rel_res, hipStream_t st) {
    if (o->prec == CHAFF_C64)
        return solve_impl<c64, c64>(c, o, (const c64*)Z, (const c64*)Pinv, k_hat, e_hat, s, (c128*)X, ws,
                                    ws_bytes, st_out, rel_res, st);
    return solve_impl<c128, c128>(c, o, (const c128*)Z, (const c128*)Pinv, k_hat, e_hat, s, (c128*)X, ws,
                                  ws_bytes, st_out, rel_res, st);
}

// Time every product variant on the caller's Z, X, Y and record the fastest.
chaff_status autotune(Cloud* c, chaff_prec prec, const void* Z, void* X, void* Y, int64_t s, int32_t* best,
                      double* best_ms, hipStream_t st) {
    TuneEntry t{};
    t.nb = NB;
    t.n = c->n;
    t.nnzb = c->nnzb;
    t.s = s;
    t.prec = prec;
    hipEvent_t a, b;
    CHAFF_HIP(hipEventCreate(&a));
    CHAFF_HIP(hipEventCreate(&b));
    double bms = 1e300;
    int bv = default_variant(s);
    for (int v = 0; v <= 7; ++v) {
        for (int rep = 0; rep < 7; ++rep) {
            if (rep == 2) CHAFF_HIP(hipEventRecord(a, st));
            chaff_status r = spmm_public(c, prec, Z, X, Y, s, v, st);
            if (r != CHAFF_OK) {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
                return r;
            }
        }
        CHAFF_HIP(hipEventRecord(b, st));
        CHAFF_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        CHAFF_HIP(hipEventElapsedTime(&ms, a, b));
        t.ms[v] = ms / 5.0;
        if (t.ms[v] < bms) {
            bms = t.ms[v];
            bv = v;
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    t.best = bv;
    record_tuning(t);
    if (best) *best = bv;
    if (best_ms) *best_ms = bms;
    return CHAFF_OK;
}

chaff_status excitation(Cloud* c, const double* k_hat, const double* e_hat, int64_t s, void* U, hipStream_t st) {
    const double k = 2.0 * PI_K / c->wavelength;
    hipLaunchKernelGGL(k_excitation, dim3(blocks_for(c->n * s)), dim3(256), 0, st, (const Wire*)c->wires,
                       (const int32_t*)c->perm, c->n, k_hat, e_hat, s, k, (c128*)U, (c64*)nullptr);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

}  // namespace CHAFF_KNS
}  // namespace chaff
