// Cluster block-Jacobi preconditioner: the block-Jacobi preconditioner of
// Sec. II-B (inverse diagonal blocks) taken over groups of nearby wires
// instead of single wires, so that the strongest near-field couplings are
// inverted exactly rather than left to the Krylov iteration.
//
// Clusters are runs of CLW = 8 consecutive wires of one cloud in the internal
// order.  The neighbour search sorts wires by (cloud, Morton code of their
// cell, caller index), so a run is a compact group of neighbours; the last
// cluster of a cloud may be shorter.  A cluster's block is the inverse of its
// (7 w x 7 w) diagonal submatrix of the sparsified Z (eq. 9), padded to
// 56 x 56 with the identity.  Z is complex symmetric, hence so is every block,
// and COCG stays valid.
//
// Design (gfx950):
//  * build: one workgroup per cluster.  The cluster's Z blocks are located
//    through the CSR pattern, then Gauss-Jordan with partial pivoting runs in
//    FP64 with the 56 x 56 matrix held in registers (each of the 256 lanes
//    owns a 2 x 7 tile).  Only the pivot column and the scaled pivot row pass
//    through LDS (double-buffered, three barriers a step); rows are never
//    moved: the pivot order is recorded and undone when the inverse is written,
//    through an LDS staging tile so that the stores are coalesced;
//  * apply: one workgroup per cluster and RHS tile; the cluster's rows of X
//    are staged in LDS, and for 64-column tiles each wave forms 14 rows with
//    wave-uniform reads of the block.
#include "precond.hpp"

#include "prof.hpp"

#include <algorithm>
#include <type_traits>

namespace chaff {

int64_t cluster_count(const Cloud* c) {
    int64_t n = 0;
    for (int k = 0; k < c->n_clouds; ++k) n += (c->cloud_off[k + 1] - c->cloud_off[k] + CLW - 1) / CLW;
    return n;
}

size_t cluster_table_bytes(int64_t n_cl) { return align_up((size_t)n_cl * sizeof(ClusterEntry), 256); }

size_t cluster_buffer_bytes(const Cloud* c, chaff_prec prec) {
    const int64_t n_cl = cluster_count(c);
    return cluster_table_bytes(n_cl) + (size_t)n_cl * CLR2 * (prec == CHAFF_C64 ? sizeof(c64) : sizeof(c128));
}

namespace {

constexpr int GJ_TC = 8;    // column classes of the register tile: columns tc + 8 m, m < 7
constexpr int GJ_TR = 32;   // row classes: rows tr and tr + 32
static_assert(GJ_TC * GJ_TR == 256, "one tile per lane of a 256-lane workgroup");
static_assert(GJ_TC * 7 == CLR && GJ_TR * 2 >= CLR, "tiles cover the block");

__global__ void k_clear_flag(int32_t* __restrict__ flag) {
    if (threadIdx.x == 0) flag[0] = 0;
}

template <typename CZ>
__global__ __launch_bounds__(256) void k_cluster_build(const ClusterEntry* __restrict__ tab,
                                                       const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx,
                                                       const CZ* __restrict__ Z, CZ* __restrict__ M,
                                                       int32_t* __restrict__ status) {
    __shared__ int64_t blk[CLW][CLW];   // block index of (wire a, wire b) of the cluster, -1 if not stored
    __shared__ c128 colk[2][CLR];
    __shared__ c128 rowp[2][CLR];
    __shared__ c128 pinv[2];
    __shared__ int32_t pidx[2];
    __shared__ int32_t piv[CLR], ipiv[CLR], used[CLR];
    __shared__ CZ stage[CLR2];
    const ClusterEntry ce = tab[blockIdx.x];
    const int t = threadIdx.x;
    if (t < CLW * CLW) blk[t / CLW][t % CLW] = -1;
    if (t < CLR) used[t] = 0;
    __syncthreads();
    if (t < ce.nw) {
        const int64_t i = (int64_t)ce.w0 + t;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col_idx[e];
            if (j >= ce.w0 && j < ce.w0 + ce.nw) blk[t][j - ce.w0] = e;
        }
    }
    __syncthreads();

    const int tc = t % GJ_TC, tr = t / GJ_TC;
    c128 B[2][7];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int r = tr + GJ_TR * a;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const int cc = tc + GJ_TC * m;
            c128 v = {0.0, 0.0};
            if (r < CLR) {
                const int wa = r / NB, wb = cc / NB;
                if (wa < ce.nw && wb < ce.nw) {
                    const int64_t e = blk[wa][wb];
                    if (e >= 0) v = ccast<c128>(Z[e * NB2 + (r % NB) * NB + (cc % NB)]);
                } else if (r == cc) {
                    v = c128{1.0, 0.0};
                }
            }
            B[a][m] = v;
        }
    }

    for (int k = 0; k < CLR; ++k) {
        const int buf = k & 1;
        if (tc == k % GJ_TC) {   // owners of column k publish it
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                if (m == k / GJ_TC) {
                    colk[buf][tr] = B[0][m];
                    if (tr + GJ_TR < CLR) colk[buf][tr + GJ_TR] = B[1][m];
                }
            }
        }
        __syncthreads();
        if (t < 64) {   // pivot: largest |a_rk| among rows not yet used, lowest row on ties
            double mag = -1.0;
            int idx = t;
            if (t < CLR && !used[t]) {   // every unused row competes (a NaN as 0): the winner is one of them
                const c128 v = colk[buf][t];
                mag = v.re * v.re + v.im * v.im;
                if (!(mag >= 0.0)) mag = 0.0;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double om = __shfl_xor(mag, off, 64);
                const int oi = __shfl_xor(idx, off, 64);
                if (om > mag || (om == mag && oi < idx)) {
                    mag = om;
                    idx = oi;
                }
            }
            if (t == 0) {
                const c128 d = colk[buf][idx];
                const double m2 = d.re * d.re + d.im * d.im;
                c128 inv = {0.0, 0.0};
                if (m2 > 0.0 && isfinite(m2)) inv = c128{d.re / m2, -d.im / m2};
                else atomicOr(status, 1);
                piv[k] = idx;
                used[idx] = 1;
                pidx[buf] = idx;
                pinv[buf] = inv;
            }
        }
        __syncthreads();
        const int p = pidx[buf];
        const c128 inv = pinv[buf];
#pragma unroll
        for (int a = 0; a < 2; ++a) {   // owners of pivot row p publish it, scaled
            if (tr + GJ_TR * a == p) {
#pragma unroll
                for (int m = 0; m < 7; ++m) {
                    const int cc = tc + GJ_TC * m;
                    rowp[buf][cc] = (cc == k) ? inv : cmul(B[a][m], inv);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int r = tr + GJ_TR * a;
            if (r >= CLR) continue;
            const c128 f = colk[buf][r];
            const c128 nf = {-f.re, -f.im};
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                const int cc = tc + GJ_TC * m;
                const c128 rp = rowp[buf][cc];
                if (r == p) {
                    B[a][m] = rp;
                } else {
                    c128 v = (cc == k) ? c128{0.0, 0.0} : B[a][m];
                    cfma(v, nf, rp);
                    B[a][m] = v;
                }
            }
        }
    }
    // Row p_k of the working array is row k of the inverse of the row-permuted
    // matrix; undoing the permutation puts entry (r, c) at (ipiv[r], piv[c]).
    __syncthreads();
    if (t < CLR) ipiv[piv[t]] = t;
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int r = tr + GJ_TR * a;
        if (r >= CLR) continue;
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            const int cc = tc + GJ_TC * m;
            stage[ipiv[r] * CLR + piv[cc]] = ccast<CZ>(B[a][m]);
        }
    }
    __syncthreads();
    CZ* out = M + (int64_t)blockIdx.x * CLR2;
    for (int e = t; e < CLR2; e += 256) out[e] = stage[e];
}

template <typename CZ, typename CI, typename CO, bool ACC, int ST>
__global__ __launch_bounds__(256) void k_cluster_apply(const ClusterEntry* __restrict__ tab, const CZ* __restrict__ M,
                                                       const CI* __restrict__ X, CO* __restrict__ Y, int64_t s) {
    using A = typename std::conditional<sizeof(CZ) == 16 || sizeof(CI) == 16 || sizeof(CO) == 16, double,
                                        float>::type;
    constexpr int NSUB = 256 / ST;
    constexpr int RPT = (CLR + NSUB - 1) / NSUB;
    constexpr bool FULL = NSUB * RPT == CLR;
    constexpr bool STAGED = sizeof(CZ) == sizeof(c64);   // complex64 blocks are staged in LDS (25 KB)
    __shared__ __align__(16) cplx<A> xs[CLR * ST];
    __shared__ __align__(16) CZ ms[STAGED ? CLR2 : 2];
    const ClusterEntry ce = tab[blockIdx.x];
    const int col = threadIdx.x % ST;
    const int rsub = ST == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / ST);
    const int64_t r = (int64_t)blockIdx.y * ST + col;
    const int nr = ce.nw * NB;
    const int64_t row0 = (int64_t)ce.w0 * NB;
    const CZ* mb = M + (int64_t)blockIdx.x * CLR2;
    if (STAGED) stage_block<CZ, 256>(ms, mb);
    for (int rho = (int)(threadIdx.x / ST); rho < CLR; rho += NSUB) {
        cplx<A> v = {0, 0};
        if (rho < nr && r < s) v = ccast<cplx<A>>(X[(row0 + rho) * s + r]);
        xs[rho * ST + col] = v;
    }
    __syncthreads();
    if (r >= s) return;
    cplx<A> acc[RPT];
    cluster_rows<A, CZ, ST, RPT, FULL, STAGED>(ms, mb, xs, col, rsub, acc);
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rho = rsub * RPT + j;
        if (rho < nr) {
            const int64_t o = (row0 + rho) * s + r;
            if (ACC) {
                CO y = Y[o];
                y.re += acc[j].re;
                y.im += acc[j].im;
                Y[o] = y;
            } else {
                Y[o] = ccast<CO>(acc[j]);
            }
        }
    }
}

template <typename CZ, typename CI, typename CO, bool ACC>
void apply_dispatch(int64_t n_cl, const ClusterEntry* tab, const CZ* M, const CI* X, CO* Y, int64_t s,
                    hipStream_t st) {
    // 64-column tiles of complex doubles would not fit beside the staged block
    constexpr int WMAX = (sizeof(CZ) == 16 || sizeof(CI) == 16 || sizeof(CO) == 16) ? 32 : 64;
    int w = 1;
    while (w < s && w < WMAX) w <<= 1;
    const dim3 grid((unsigned)n_cl, (unsigned)((s + w - 1) / w));
    switch (w) {
        case 1: hipLaunchKernelGGL((k_cluster_apply<CZ, CI, CO, ACC, 1>), grid, dim3(256), 0, st, tab, M, X, Y, s); break;
        case 2: hipLaunchKernelGGL((k_cluster_apply<CZ, CI, CO, ACC, 2>), grid, dim3(256), 0, st, tab, M, X, Y, s); break;
        case 4: hipLaunchKernelGGL((k_cluster_apply<CZ, CI, CO, ACC, 4>), grid, dim3(256), 0, st, tab, M, X, Y, s); break;
        case 8: hipLaunchKernelGGL((k_cluster_apply<CZ, CI, CO, ACC, 8>), grid, dim3(256), 0, st, tab, M, X, Y, s); break;
        case 16: hipLaunchKernelGGL((k_cluster_apply<CZ, CI, CO, ACC, 16>), grid, dim3(256), 0, st, tab, M, X, Y, s); break;
        case 32: hipLaunchKernelGGL((k_cluster_apply<CZ, CI, CO, ACC, 32>), grid, dim3(256), 0, st, tab, M, X, Y, s); break;
        default:
            if constexpr (WMAX == 64)
                hipLaunchKernelGGL((k_cluster_apply<CZ, CI, CO, ACC, 64>), grid, dim3(256), 0, st, tab, M, X, Y, s);
            break;
    }
}

template <typename CZ>
const CZ* blocks_of(const void* M, int64_t n_cl) {
    return reinterpret_cast<const CZ*>(static_cast<const char*>(M) + cluster_table_bytes(n_cl));
}

}  // namespace

chaff_status cluster_apply_launch(const Cloud* c, chaff_prec prec, const void* M, const void* X, bool x64, void* Y,
                                  bool y64, bool accumulate, int64_t s, hipStream_t st, const char* prof_name) {
    const int64_t n_cl = cluster_count(c);
    if (n_cl == 0) return CHAFF_OK;
    const ClusterEntry* tab = static_cast<const ClusterEntry*>(M);
    const size_t zb = prec == CHAFF_C64 ? sizeof(c64) : sizeof(c128);
    ProfScope ps(prof_name, st,
                 (double)n_cl * CLR2 * zb + (double)c->n * NB * s * ((x64 ? 16.0 : zb) + (y64 ? 16.0 : zb) * (accumulate ? 2 : 1)));
    if (prec == CHAFF_C64) {
        const c64* Mb = blocks_of<c64>(M, n_cl);
        if (!x64 && !y64 && !accumulate)
            apply_dispatch<c64, c64, c64, false>(n_cl, tab, Mb, (const c64*)X, (c64*)Y, s, st);
        else if (!x64 && y64 && accumulate)
            apply_dispatch<c64, c64, c128, true>(n_cl, tab, Mb, (const c64*)X, (c128*)Y, s, st);
        else if (x64 && y64 && !accumulate)
            apply_dispatch<c64, c128, c128, false>(n_cl, tab, Mb, (const c128*)X, (c128*)Y, s, st);
        else
            return fail(CHAFF_EINVAL, "internal: unsupported cluster apply combination");
    } else {
        if (!(x64 && y64)) return fail(CHAFF_EINVAL, "internal: complex128 cluster apply needs complex128 vectors");
        const c128* Mb = blocks_of<c128>(M, n_cl);
        if (accumulate)
            apply_dispatch<c128, c128, c128, true>(n_cl, tab, Mb, (const c128*)X, (c128*)Y, s, st);
        else
            apply_dispatch<c128, c128, c128, false>(n_cl, tab, Mb, (const c128*)X, (c128*)Y, s, st);
    }
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status cluster_precond(Cloud* c, chaff_prec prec, const void* Z, void* M, hipStream_t st) {
    const int64_t n_cl = cluster_count(c);
    if (n_cl == 0) return CHAFF_OK;
    std::vector<ClusterEntry> tab((size_t)n_cl);
    int64_t k = 0;
    for (int cl = 0; cl < c->n_clouds; ++cl)
        for (int64_t w0 = c->cloud_off[cl]; w0 < c->cloud_off[cl + 1]; w0 += CLW)
            tab[k++] = ClusterEntry{(int32_t)w0, (int32_t)std::min<int64_t>(CLW, c->cloud_off[cl + 1] - w0)};
    CHAFF_HIP(hipMemcpyAsync(M, tab.data(), tab.size() * sizeof(ClusterEntry), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, c->d_status);
    CHAFF_LAUNCH_CHECK();
    {
        ProfScope ps("cluster_build", st, (double)n_cl * CLR * (8.0 * CLR * CLR), true);
        const ClusterEntry* dt = static_cast<const ClusterEntry*>(M);
        char* blocks = static_cast<char*>(M) + cluster_table_bytes(n_cl);
        if (prec == CHAFF_C64)
            hipLaunchKernelGGL((k_cluster_build<c64>), dim3((unsigned)n_cl), dim3(256), 0, st, dt,
                               (const int64_t*)c->row_ptr, (const int32_t*)c->col_idx, (const c64*)Z, (c64*)blocks,
                               c->d_status);
        else
            hipLaunchKernelGGL((k_cluster_build<c128>), dim3((unsigned)n_cl), dim3(256), 0, st, dt,
                               (const int64_t*)c->row_ptr, (const int32_t*)c->col_idx, (const c128*)Z,
                               (c128*)blocks, c->d_status);
        CHAFF_LAUNCH_CHECK();
    }
    int32_t flag = 0;
    CHAFF_HIP(hipMemcpyAsync(&flag, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipStreamSynchronize(st));   // also keeps the host table alive until copied
    if (flag) return fail(CHAFF_ESINGULAR, "a cluster block has a zero pivot");
    return CHAFF_OK;
}

chaff_status cluster_check_table(const Cloud* c, const void* M, hipStream_t st) {
    const int64_t n_cl = cluster_count(c);
    if (n_cl == 0) return CHAFF_OK;
    ClusterEntry got[2];
    const ClusterEntry* tab = static_cast<const ClusterEntry*>(M);
    CHAFF_HIP(hipMemcpyAsync(&got[0], tab, sizeof(ClusterEntry), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipMemcpyAsync(&got[1], tab + (n_cl - 1), sizeof(ClusterEntry), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipStreamSynchronize(st));
    int last = c->n_clouds - 1;
    while (last > 0 && c->cloud_off[last] == c->cloud_off[last + 1]) --last;
    int first = 0;
    while (first < last && c->cloud_off[first] == c->cloud_off[first + 1]) ++first;
    const int64_t nl = c->cloud_off[last + 1] - c->cloud_off[last];
    const ClusterEntry e0{(int32_t)c->cloud_off[first],
                          (int32_t)std::min<int64_t>(CLW, c->cloud_off[first + 1] - c->cloud_off[first])};
    const ClusterEntry e1{(int32_t)(c->cloud_off[last] + (nl - 1) / CLW * CLW),
                          (int32_t)(nl - (nl - 1) / CLW * CLW)};
    if (got[0].w0 != e0.w0 || got[0].nw != e0.nw || got[1].w0 != e1.w0 || got[1].nw != e1.nw)
        return fail(CHAFF_EINVAL, "the preconditioner buffer is not a cluster preconditioner of this cloud "
                                  "(build it with chaff_cluster_precond)");
    return CHAFF_OK;
}

chaff_status cluster_apply_public(Cloud* c, chaff_prec prec, const void* M, const void* X, void* Y, int64_t s,
                                  hipStream_t st) {
    chaff_status ck = cluster_check_table(c, M, st);
    if (ck != CHAFF_OK) return ck;
    const bool w = prec == CHAFF_C128;
    return cluster_apply_launch(c, prec, M, X, w, Y, w, false, s, st, "cluster_apply");
}

}  // namespace chaff
