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


// ==================================================================== neighbourhood inverse
//
// Design (gfx950):
//  * selection: one lane per wire walks its row of the pattern (all near-set
//    neighbours) and keeps the size - 1 nearest in a sorted register list
//    (FP64 squared centroid distance formed as in the near-set test, ties to
//    the lower caller index);
//  * build: one wave per wire.  Lane r owns row r of the local system
//    [A | E] (A the neighbourhood's 7 m x 7 m submatrix of Z padded to
//    7 KM rows with the identity, E the wire's own 7 unit columns) in FP32
//    registers; Gauss-Jordan with partial pivoting: the pivot row is chosen
//    by a wave reduction over the unused rows, normalised by its lane, and
//    broadcast column by column with readlane, so no row is ever moved
//    (an LDS broadcast of the pivot row measured slower: 40.6 against 30.9 ms
//    at C5, eight wires, as its extra registers leave two waves per SIMD).  The
//    pivot row of unknown u ends holding row u of A^-1 E, i.e. column u of
//    p's row block of A^-1 (A is complex symmetric), which is written at the
//    block position of (p, member) in Z's pattern;
//  * symmetrisation: one wave per unique pair (and per diagonal block), lane
//    = block entry: M_pq = (raw_pq + raw_qp^T) / 2, M_qp = M_pq^T.
size_t nbhd_table_bytes(int64_t n, int size) { return align_up((size_t)n * size * sizeof(int32_t), 256); }

size_t nbhd_buffer_bytes(const Cloud* c, chaff_prec prec, int size) {
    return nbhd_blocks_offset(c->n, size) + (size_t)c->nnzb * NB2 * (prec == CHAFF_C64 ? sizeof(c64) : sizeof(c128));
}

namespace {

constexpr int NBH_WAVES = 4;

__global__ __launch_bounds__(256) void k_zero_words(uint32_t* __restrict__ a, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        a[t] = 0u;
}

__global__ __launch_bounds__(256) void k_nbhd_select(int64_t n, int size, const Wire* __restrict__ wires,
                                                     const int32_t* __restrict__ perm,
                                                     const int64_t* __restrict__ row_ptr,
                                                     const int32_t* __restrict__ col_idx, int32_t* __restrict__ nbt) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int L = NBH_MAX - 1;
    double bd[L];
    int32_t bk[L], bj[L];
#pragma unroll
    for (int t = 0; t < L; ++t) {
        bd[t] = INFINITY;
        bk[t] = 0x7fffffff;
        bj[t] = -1;
    }
    const Wire wi = wires[i];
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int32_t j = col_idx[e];
        if (j == i) continue;
        const Wire& wj = wires[j];
        const double dx = wj.cx - wi.cx;
        const double dy = wj.cy - wi.cy;
        const double dz = wj.cz - wi.cz;
        const double xx = dx * dx;
        const double yy = dy * dy;
        const double zz = dz * dz;
        double d2 = xx + yy;
        d2 = d2 + zz;
        double cd = d2;
        int32_t ck = perm[j], cj = j;
        // one insertion pass: the list stays sorted by (distance, caller index)
#pragma unroll
        for (int t = 0; t < L; ++t) {
            const bool lt = cd < bd[t] || (cd == bd[t] && ck < bk[t]);
            const double td = bd[t];
            const int32_t tk = bk[t], tj = bj[t];
            bd[t] = lt ? cd : td;
            bk[t] = lt ? ck : tk;
            bj[t] = lt ? cj : tj;
            cd = lt ? td : cd;
            ck = lt ? tk : ck;
            cj = lt ? tj : cj;
        }
    }
    int32_t* out = nbt + i * size;
    out[0] = (int32_t)i;
#pragma unroll
    for (int t = 0; t < L; ++t)
        if (t + 1 < size) out[t + 1] = bj[t];
}

// Wave arg-max of a non-negative magnitude over the lanes still competing:
// each lane forms the key (magnitude bits with the low 6 cleared) | (63 - lane)
// (float bits order like the magnitudes; the lowest lane wins a tie), the
// keys are reduced with DPP moves inside each row of 16 lanes and the four
// row maxima read back to the scalar unit.  The magnitudes compared keep 17
// of their 23 fraction bits, so the pivot is the largest to 2^-17 — still a
// partial pivot.
__device__ __forceinline__ int pivot_lane(bool used, float mag, int lane) {
    if (!(mag >= 0.f)) mag = 0.f;
    uint32_t key = used ? 0u : ((__float_as_uint(mag) & ~63u) | (uint32_t)(63 - lane));
    // quad_perm [1,0,3,2] (lane ^ 1), quad_perm [2,3,0,1] (lane ^ 2), row_half_mirror, row_mirror
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0xB1, 0xF, 0xF, false));
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x4E, 0xF, 0xF, false));
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x141, 0xF, 0xF, false));
    key = max(key, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x140, 0xF, 0xF, false));
    const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, 0);
    const uint32_t k1 = (uint32_t)__builtin_amdgcn_readlane((int)key, 16);
    const uint32_t k2 = (uint32_t)__builtin_amdgcn_readlane((int)key, 32);
    const uint32_t k3 = (uint32_t)__builtin_amdgcn_readlane((int)key, 48);
    const uint32_t best = max(max(k0, k1), max(k2, k3));
    return 63 - (int)(best & 63u);
}

template <typename CZ, int KM>
__global__ __launch_bounds__(64 * NBH_WAVES) void k_nbhd_build(int64_t n, int size, const int32_t* __restrict__ nbt,
                                                               const int64_t* __restrict__ row_ptr,
                                                               const int32_t* __restrict__ col_idx,
                                                               const CZ* __restrict__ Z, CZ* __restrict__ M,
                                                               int32_t* __restrict__ status) {
    constexpr int NR = NB * KM;   // rows of the padded local system
    constexpr int NC = NR + NB;   // its columns and the wire's own unit vectors
    static_assert(NR <= 64 && KM * KM <= 64, "one lane per row and per block of the local system");
    __shared__ int64_t pos_s[NBH_WAVES][KM * KM];
    const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
    const int64_t i = (int64_t)blockIdx.x * NBH_WAVES + w;
    if (i >= n) return;   // wave-uniform; the waves of a workgroup never wait for each other
    // members in the order of the local system: the neighbours first, the wire
    // itself last (its unit columns then stay untouched until its own block)
    int32_t raw[KM], mem[KM];
    int m = 0;
#pragma unroll
    for (int s = 0; s < KM; ++s) {
        raw[s] = s < size ? nbt[i * size + s] : -1;
        m += raw[s] >= 0 ? 1 : 0;
    }
#pragma unroll
    for (int s = 0; s < KM; ++s) mem[s] = s + 1 < m ? raw[s + 1] : (s + 1 == m ? raw[0] : -1);
    const int own = NB * (m - 1);   // first row of the wire's own block
    // block position of (member a, member b) in Z's pattern, -1 if the pair is not near
    if (lane < KM * KM) {
        const int a = lane / KM, b = lane % KM;
        int64_t p = -1;
        if (a < m && b < m) {
            const int32_t row = mem[a], target = mem[b];
            for (int64_t e = row_ptr[row]; e < row_ptr[row + 1]; ++e)
                if (col_idx[e] == target) p = e;
        }
        pos_s[w][lane] = p;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const int ra = lane / NB, rq = lane % NB;
    c64 A[NC];
#pragma unroll
    for (int b = 0; b < KM; ++b) {
        int64_t p = -1;
        if (lane < NR && ra < m && b < m) p = pos_s[w][ra * KM + b];
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int col = NB * b + c;
            c64 v = {0.f, 0.f};
            if (p >= 0)
                v = ccast<c64>(Z[p * NB2 + rq * NB + c]);
            else if (lane < NR && ra >= m && lane == col)
                v = c64{1.f, 0.f};   // padding rows and columns: the identity
            A[col] = v;
        }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) A[NR + c] = c64{lane == own + c ? 1.f : 0.f, 0.f};

    // Gauss-Jordan over the 7 m columns of the real system (padding rows keep
    // their identity entries and never compete for a pivot).  Rows are not
    // normalised: the pivot row of column k keeps its pivot d_k, the other rows
    // subtract (a_rk / d_k) times it, and at the end row piv(u) holds d_u in
    // column u, zeros in every other column and d_u x_u in the unit columns.
    // Columns are walked block by block: block kb's 7 columns are copied once
    // into T (static indices from then on); columns of earlier blocks are never
    // read again, so only T, the later blocks and the unit columns change.
    // The pivots of the neighbours' columns are taken among the neighbours'
    // rows only (partial pivoting on the leading block, whose Schur complement
    // is the wire's own block): every pivot row then has zero unit columns
    // until the last block, so those columns are left alone until then.
    const int nr = NB * m;
    bool used = lane >= nr;
    int my_u = -1;
    c64 my_d = {1.f, 0.f};
    bool bad = false;
    for (int kb = 0; kb < m; ++kb) {
        c64 T[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) T[c] = A[c];
#pragma unroll
        for (int b = 1; b < KM; ++b)
            if (b == kb) {
#pragma unroll
                for (int c = 0; c < NB; ++c) T[c] = A[NB * b + c];
            }
#pragma unroll
        for (int kc = 0; kc < NB; ++kc) {
            const c64 v = T[kc];
            // pivot: the largest |a_rk| among rows not yet used (NaN counts as 0)
            const bool own_block = kb == m - 1;   // wave-uniform
            const int piv = pivot_lane(used || (!own_block && lane >= own), v.re * v.re + v.im * v.im, lane);
            const c64 pv = {__int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.re), piv)),
                            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.im), piv))};
            const float d = pv.re * pv.re + pv.im * pv.im;
            c64 inv = {0.f, 0.f};
            if (d > 0.f && d < INFINITY) inv = c64{pv.re / d, -pv.im / d};
            else bad = true;
            if (lane == piv) {
                used = true;
                my_u = NB * kb + kc;
                my_d = pv;
            }
            const c64 l = (lane == piv || lane >= NR) ? c64{0.f, 0.f} : cmul(v, inv);
            auto elim = [&](c64& a) {
                const c64 pj = {__int_as_float(__builtin_amdgcn_readlane(__float_as_int(a.re), piv)),
                                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a.im), piv))};
                a.re = fmaf(-l.re, pj.re, a.re);
                a.re = fmaf(l.im, pj.im, a.re);
                a.im = fmaf(-l.re, pj.im, a.im);
                a.im = fmaf(-l.im, pj.re, a.im);
            };
#pragma unroll
            for (int c = kc + 1; c < NB; ++c) elim(T[c]);
#pragma unroll
            for (int b = 1; b < KM; ++b)
                if (b > kb) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) elim(A[NB * b + c]);
                }
            if (own_block) {
#pragma unroll
                for (int c = 0; c < NB; ++c) elim(A[NR + c]);
            }
        }
    }
    // the pivot row of unknown u holds d_u times row u of A^-1 E: raw_{p, mem[s]}[c][a] with u = 7 s + a
    if (my_u >= 0) {
        const int s = my_u / NB, a = my_u % NB;
        const float dd = my_d.re * my_d.re + my_d.im * my_d.im;
        const c64 id = dd > 0.f ? c64{my_d.re / dd, -my_d.im / dd} : c64{0.f, 0.f};
        if (s < m) {
            const int64_t p = pos_s[w][(m - 1) * KM + s];   // (p, mem[s]) in row p
#pragma unroll
            for (int c = 0; c < NB; ++c) M[p * NB2 + c * NB + a] = ccast<CZ>(cmul(A[NR + c], id));
        }
    }
    if (bad && lane == 0) status[0] = 1;
}

template <typename CZ>
__global__ __launch_bounds__(256) void k_nbhd_symm(int64_t n_pairs, const Pair* __restrict__ pairs, int64_t n,
                                                   const int64_t* __restrict__ diag_pos, CZ* __restrict__ M) {
    using R = typename real_of<CZ>::type;
    const int64_t u = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;   // one wave per unit
    const int e = (int)(threadIdx.x & 63);
    if (u >= n_pairs + n || e >= NB2) return;
    const int r = e / NB, c = e % NB, et = c * NB + r;
    if (u < n_pairs) {
        const Pair pr = pairs[u];
        const CZ a = M[pr.pos_ij * NB2 + e], b = M[pr.pos_ji * NB2 + et];
        const CZ v = {(a.re + b.re) * (R)0.5, (a.im + b.im) * (R)0.5};
        M[pr.pos_ij * NB2 + e] = v;    // M_pq[r][c]
        M[pr.pos_ji * NB2 + et] = v;   // M_qp[c][r]
    } else {
        const int64_t p = diag_pos[u - n_pairs];
        const CZ a = M[p * NB2 + e], b = M[p * NB2 + et];   // every lane reads before any writes (one wave)
        M[p * NB2 + e] = CZ{(a.re + b.re) * (R)0.5, (a.im + b.im) * (R)0.5};
    }
}

template <typename CZ>
void nbhd_build_launch(Cloud* c, int size, const int32_t* nbt, const CZ* Z, CZ* M, hipStream_t st) {
    const unsigned g = (unsigned)((c->n + NBH_WAVES - 1) / NBH_WAVES);
#define CHAFF_NBH(KMV)                                                                                       \
    case KMV:                                                                                                \
        hipLaunchKernelGGL((k_nbhd_build<CZ, KMV>), dim3(g), dim3(64 * NBH_WAVES), 0, st, c->n, size, nbt,   \
                           (const int64_t*)c->row_ptr, (const int32_t*)c->col_idx, Z, M, c->d_status);       \
        break;
    switch (size) {   // the local system is sized for exactly `size` wires
        CHAFF_NBH(1) CHAFF_NBH(2) CHAFF_NBH(3) CHAFF_NBH(4) CHAFF_NBH(5) CHAFF_NBH(6) CHAFF_NBH(7)
        default: CHAFF_NBH(8)
    }
#undef CHAFF_NBH
}

}  // namespace

chaff_status nbhd_begin(Cloud* c, chaff_prec prec, int size, bool raw, void* M, hipStream_t st) {
    if (size < 1 || size > NBH_MAX) return fail(CHAFF_EINVAL, "neighbourhood size must be in [1, 8]");
    NbhdHeader h{};
    h.magic = NBH_MAGIC;
    h.n = c->n;
    h.nnzb = c->nnzb;
    h.size = size;
    h.prec = (int32_t)prec;
    h.raw = raw ? 1 : 0;
    CHAFF_HIP(hipMemcpyAsync(M, &h, sizeof(h), hipMemcpyHostToDevice, st));
    CHAFF_HIP(hipStreamSynchronize(st));
    if (c->n == 0) return CHAFF_OK;
    int32_t* nbt = reinterpret_cast<int32_t*>(static_cast<char*>(M) + NBH_HEADER);
    char* vals = static_cast<char*>(M) + nbhd_blocks_offset(c->n, size);
    const size_t zb = prec == CHAFF_C64 ? sizeof(c64) : sizeof(c128);
    const int64_t words = (int64_t)((size_t)c->nnzb * NB2 * zb / 4);
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<int64_t>((words + 255) / 256, 65536)), dim3(256), 0, st,
                       (uint32_t*)vals, words);
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(64), 0, st, c->d_status);
    hipLaunchKernelGGL(k_nbhd_select, dim3((unsigned)((c->n + 255) / 256)), dim3(256), 0, st, c->n, size,
                       (const Wire*)c->wires, (const int32_t*)c->perm, (const int64_t*)c->row_ptr,
                       (const int32_t*)c->col_idx, nbt);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status nbhd_symmetrise(Cloud* c, chaff_prec prec, void* vals, hipStream_t st) {
    const int64_t units = c->n_pairs + c->n;
    if (units == 0) return CHAFF_OK;
    const unsigned gs = (unsigned)((units * 64 + 255) / 256);
    if (prec == CHAFF_C64)
        hipLaunchKernelGGL((k_nbhd_symm<c64>), dim3(gs), dim3(256), 0, st, c->n_pairs, (const Pair*)c->pairs, c->n,
                           (const int64_t*)c->diag_pos, (c64*)vals);
    else
        hipLaunchKernelGGL((k_nbhd_symm<c128>), dim3(gs), dim3(256), 0, st, c->n_pairs, (const Pair*)c->pairs, c->n,
                           (const int64_t*)c->diag_pos, (c128*)vals);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

chaff_status nbhd_precond(Cloud* c, chaff_prec prec, int size, const void* Z, void* M, bool raw, hipStream_t st) {
    chaff_status s = nbhd_begin(c, prec, size, raw, M, st);
    if (s != CHAFF_OK || c->n == 0) return s;
    const int32_t* nbt = reinterpret_cast<const int32_t*>(static_cast<const char*>(M) + NBH_HEADER);
    char* vals = static_cast<char*>(M) + nbhd_blocks_offset(c->n, size);
    {
        const size_t zb = prec == CHAFF_C64 ? sizeof(c64) : sizeof(c128);
        // algorithmic work of the elimination: at every pivot each of the nr rows
        // updates the columns still live (the rest of the pivot's block, the later
        // blocks and the wire's unit columns): m NB (NB - 1) / 2 + NB^2 m (m - 1) / 2
        // + NB^2 m complex multiply-adds per row for m wires
        const double nr = (double)NB * size, m = size;
        const double cma = m * NB * (NB - 1) / 2.0 + (double)NB2 * m * (m - 1.0) / 2.0 + (double)NB2 * m;
        ProfScope ps("nbhd_build", st, ProfWork{(double)c->nnzb * NB2 * zb, (double)c->n * nr * cma * 8.0});
        if (prec == CHAFF_C64)
            nbhd_build_launch<c64>(c, size, nbt, (const c64*)Z, (c64*)vals, st);
        else
            nbhd_build_launch<c128>(c, size, nbt, (const c128*)Z, (c128*)vals, st);
        CHAFF_LAUNCH_CHECK();
    }
    if (!raw) {
        s = nbhd_symmetrise(c, prec, vals, st);
        if (s != CHAFF_OK) return s;
    }
    int32_t flag = 0;
    CHAFF_HIP(hipMemcpyAsync(&flag, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipStreamSynchronize(st));
    if (flag) return fail(CHAFF_ESINGULAR, "a neighbourhood system has a zero pivot");
    return CHAFF_OK;
}

chaff_status nbhd_header(const Cloud* c, const void* M, NbhdHeader* h, hipStream_t st) {
    CHAFF_HIP(hipMemcpyAsync(h, M, sizeof(*h), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipStreamSynchronize(st));
    if (h->magic != NBH_MAGIC || h->n != c->n || h->nnzb != c->nnzb || h->size < 1 || h->size > NBH_MAX)
        return fail(CHAFF_EINVAL, "the buffer is not a neighbourhood-inverse preconditioner buffer of this cloud "
                                  "(build it with chaff_nbhd_precond)");
    return CHAFF_OK;
}

chaff_status nbhd_check(const Cloud* c, chaff_prec prec, const void* M, int* size, hipStream_t st) {
    NbhdHeader h{};
    chaff_status s = nbhd_header(c, M, &h, st);
    if (s != CHAFF_OK) return s;
    if (h.prec != (int32_t)prec)
        return fail(CHAFF_EINVAL, "the neighbourhood-inverse preconditioner was built for the other precision");
    if (h.raw)
        return fail(CHAFF_EINVAL, "the buffer holds unsymmetrised neighbourhood rows (chaff_nbhd_raw_rows), "
                                  "not a preconditioner");
    *size = h.size;
    return CHAFF_OK;
}

}  // namespace chaff
