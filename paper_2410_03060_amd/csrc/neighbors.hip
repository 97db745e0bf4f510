// Neighbour search for the S-NFC pattern (eq. 9): keep wire pairs of one
// cloud whose centroid distance is <= d_c.
//
// Design (gfx950):
//  * a cell grid per cloud with cell side h >= d_c (slightly larger, so that
//    rounding can never put two wires within d_c more than one cell apart);
//  * wires are ordered by (cloud, Morton code of their cell) with a stable
//    hand-written LSD radix sort (8-bit digits, wave64 ballot ranking), which
//    gives the block pattern spatial locality for the sparse products;
//  * dense per-cloud tables map a linear cell index to its run of sorted wires;
//  * two passes over the 27 neighbouring cells per wire: count, exclusive scan,
//    then write the column indices in ascending order (cells are visited in
//    the order of their run start, runs are disjoint), the diagonal position
//    and the unique pair list (i < j) used by the fill.
#include "common.hpp"
#include "prof.hpp"

#include <algorithm>

namespace chaff {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint64_t spread3(uint64_t v) {  // up to 21 bits -> every third bit
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x001F00000000FFFFull;
    v = (v | (v << 16)) & 0x001F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ void cell_of(const CloudGrid& g, double x, double y, double z,
                                        int& ix, int& iy, int& iz) {
    if (g.inv_h == 0.0) {
        ix = iy = iz = 0;
        return;
    }
    double fx = floor((x - g.ox) * g.inv_h);
    double fy = floor((y - g.oy) * g.inv_h);
    double fz = floor((z - g.oz) * g.inv_h);
    ix = (int)fmin(fmax(fx, 0.0), (double)(g.nx - 1));
    iy = (int)fmin(fmax(fy, 0.0), (double)(g.ny - 1));
    iz = (int)fmin(fmax(fz, 0.0), (double)(g.nz - 1));
}

// FP64 squared centroid distance evaluated as ((dx*dx + dy*dy) + dz*dz), each
// operation rounded (no contraction), so that the host-side definition is
// reproduced bit for bit.
__device__ __forceinline__ bool within(const double* __restrict__ ci, const double* __restrict__ cj,
                                       double dc2) {
#pragma clang fp contract(off)
    double dx = cj[0] - ci[0];
    double dy = cj[1] - ci[1];
    double dz = cj[2] - ci[2];
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double s = xx + yy;
    s = s + zz;
    return s <= dc2;
}

// ------------------------------------------------------------------ bbox + validation

constexpr int BBOX_BLOCKS = 64;

__global__ void k_bbox(const double* __restrict__ center, const double* __restrict__ tangent,
                       const double* __restrict__ length, const double* __restrict__ radius,
                       const int64_t* __restrict__ cloud_off, double* __restrict__ part,
                       int32_t* __restrict__ bad, int nseg) {
    const int c = blockIdx.y;
    const int64_t w0 = cloud_off[c], w1 = cloud_off[c + 1];
    double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    int nbad = 0;
    for (int64_t p = w0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < w1;
         p += (int64_t)gridDim.x * blockDim.x) {
        double x = center[3 * p], y = center[3 * p + 1], z = center[3 * p + 2];
        double tx = tangent[3 * p], ty = tangent[3 * p + 1], tz = tangent[3 * p + 2];
        double L = length[p], a = radius[p];
        double tn = tx * tx + ty * ty + tz * tz;
        bool ok = isfinite(x) && isfinite(y) && isfinite(z) && fabs(tn - 1.0) <= 1e-10 &&
                  isfinite(L) && L > 0.0 && isfinite(a) && a > 0.0 && a < L / nseg;
        nbad += ok ? 0 : 1;
        if (ok) {
            mn[0] = fmin(mn[0], x); mn[1] = fmin(mn[1], y); mn[2] = fmin(mn[2], z);
            mx[0] = fmax(mx[0], x); mx[1] = fmax(mx[1], y); mx[2] = fmax(mx[2], z);
        }
    }
    __shared__ double red[6][256];
    __shared__ int redbad[256];
    for (int d = 0; d < 3; ++d) {
        red[d][threadIdx.x] = mn[d];
        red[3 + d][threadIdx.x] = mx[d];
    }
    redbad[threadIdx.x] = nbad;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int d = 0; d < 3; ++d) {
                red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + s]);
                red[3 + d][threadIdx.x] = fmax(red[3 + d][threadIdx.x], red[3 + d][threadIdx.x + s]);
            }
            redbad[threadIdx.x] += redbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = part + ((int64_t)c * gridDim.x + blockIdx.x) * 6;
        for (int d = 0; d < 6; ++d) o[d] = red[d][0];
        if (redbad[0]) atomicAdd(bad, redbad[0]);
    }
}

// ------------------------------------------------------------------ keys

__global__ void k_keys(const double* __restrict__ center, const CloudGrid* __restrict__ grids,
                       int dim_bits, uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
    const int c = blockIdx.y;
    const CloudGrid g = grids[c];
    for (int64_t p = g.w0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < g.w1;
         p += (int64_t)gridDim.x * blockDim.x) {
        int ix, iy, iz;
        cell_of(g, center[3 * p], center[3 * p + 1], center[3 * p + 2], ix, iy, iz);
        uint64_t m = spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2);
        keys[p] = ((uint64_t)c << (3 * dim_bits)) | m;
        vals[p] = (int32_t)p;
    }
}

// ------------------------------------------------------------------ radix sort (stable LSD)

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

__global__ void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                          int32_t* __restrict__ hist, int n_tiles) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_ITEMS; ++k) {
        int64_t idx = base + k * RS_THREADS + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Scatter one tile.  Rounds of 256 consecutive keys keep the input order:
// inside a wave the rank among equal digits comes from 8 ballots, across
// waves from per-wave digit counts in LDS, across rounds from running counts.
__global__ void k_rs_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                             uint64_t* __restrict__ kout, int32_t* __restrict__ vout, int64_t n,
                             int shift, const int32_t* __restrict__ offs, int n_tiles) {
    __shared__ int32_t running[256];
    __shared__ int32_t wcount[RS_THREADS / 64][256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    running[threadIdx.x] = offs[(int64_t)threadIdx.x * n_tiles + blockIdx.x];
    for (int w = 0; w < RS_THREADS / 64; ++w) wcount[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int k = 0; k < RS_ITEMS; ++k) {
        int64_t idx = base + k * RS_THREADS + threadIdx.x;
        bool valid = idx < n;
        uint64_t key = valid ? kin[idx] : 0;
        int32_t val = valid ? vin[idx] : 0;
        int d = valid ? (int)((key >> shift) & 0xFF) : 256;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot(valid && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        int rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcount[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = running[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcount[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < RS_THREADS / 64; ++w) {
            tot += wcount[w][threadIdx.x];
            wcount[w][threadIdx.x] = 0;
        }
        running[threadIdx.x] += tot;
        __syncthreads();
    }
}

// ------------------------------------------------------------------ exclusive scans

constexpr int SCAN_BLOCK = 1024;

template <typename TI, typename TO>
__global__ void k_scan_block_sums(const TI* __restrict__ in, int64_t n, TO* __restrict__ sums) {
    __shared__ TO s[SCAN_BLOCK];
    int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    s[threadIdx.x] = i < n ? (TO)in[i] : (TO)0;
    __syncthreads();
    for (int st = SCAN_BLOCK / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = s[0];
}

// In-place exclusive scan of `n` values by one block (sequential over chunks).
template <typename T>
__global__ void k_scan_single(T* __restrict__ a, int64_t n, T* __restrict__ total) {
    __shared__ T s[SCAN_BLOCK];
    __shared__ T carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += SCAN_BLOCK) {
        int64_t i = base + threadIdx.x;
        T v = i < n ? a[i] : (T)0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int st = 1; st < SCAN_BLOCK; st <<= 1) {  // Hillis-Steele inclusive
            T add = threadIdx.x >= st ? s[threadIdx.x - st] : (T)0;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) a[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == SCAN_BLOCK - 1) carry += s[SCAN_BLOCK - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename TI, typename TO>
__global__ void k_scan_apply(const TI* __restrict__ in, int64_t n, const TO* __restrict__ sums,
                             TO* __restrict__ out) {
    __shared__ TO s[SCAN_BLOCK];
    int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    TO v = i < n ? (TO)in[i] : (TO)0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int st = 1; st < SCAN_BLOCK; st <<= 1) {
        TO add = threadIdx.x >= st ? s[threadIdx.x - st] : (TO)0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    if (i < n) out[i] = sums[blockIdx.x] + s[threadIdx.x] - v;
}

// exclusive scan in -> out[0..n); out[n] = total (out has n+1 entries)
template <typename TI, typename TO>
static chaff_status exclusive_scan(const TI* in, int64_t n, TO* out, TO* block_sums,
                                   hipStream_t st) {
    int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL((k_scan_block_sums<TI, TO>), dim3(nb), dim3(SCAN_BLOCK), 0, st, in, n, block_sums);
    CHAFF_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_scan_single<TO>), dim3(1), dim3(SCAN_BLOCK), 0, st, block_sums, nb, out + n);
    CHAFF_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3(nb), dim3(SCAN_BLOCK), 0, st, in, n, block_sums, out);
    CHAFF_LAUNCH_CHECK();
    return CHAFF_OK;
}

// ------------------------------------------------------------------ cells and geometry

__global__ void k_fill_i32(int32_t* __restrict__ a, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

__global__ void k_gather(const double* __restrict__ center, const double* __restrict__ tangent,
                         const double* __restrict__ length, const double* __restrict__ radius,
                         const int32_t* __restrict__ perm, const CloudGrid* __restrict__ grids,
                         int n_clouds, int64_t n, Wire* __restrict__ wires,
                         int32_t* __restrict__ iperm, int32_t* __restrict__ wire_cloud) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t p = perm[i];
        Wire w;
        w.cx = center[3 * p]; w.cy = center[3 * p + 1]; w.cz = center[3 * p + 2];
        w.tx = tangent[3 * p]; w.ty = tangent[3 * p + 1]; w.tz = tangent[3 * p + 2];
        w.len = length[p];
        w.rad = radius[p];
        wires[i] = w;
        iperm[p] = (int32_t)i;
        // clouds are contiguous in both orders: binary search on the wire ranges
        int lo = 0, hi = n_clouds - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (grids[mid].w0 <= i) lo = mid; else hi = mid - 1;
        }
        wire_cloud[i] = lo;
    }
}

__global__ void k_cells(const Wire* __restrict__ wires, const int32_t* __restrict__ wire_cloud,
                        const uint64_t* __restrict__ keys, const CloudGrid* __restrict__ grids,
                        int64_t n, int32_t* __restrict__ cell_start, int32_t* __restrict__ cell_end) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool first = (i == 0) || keys[i] != keys[i - 1];
        bool last = (i == n - 1) || keys[i] != keys[i + 1];
        if (!first && !last) continue;
        const CloudGrid g = grids[wire_cloud[i]];
        int ix, iy, iz;
        cell_of(g, wires[i].cx, wires[i].cy, wires[i].cz, ix, iy, iz);
        int64_t lin = g.cell_base + ((int64_t)iz * g.ny + iy) * g.nx + ix;
        if (first) cell_start[lin] = (int32_t)i;
        if (last) cell_end[lin] = (int32_t)(i + 1);
    }
}

// Neighbour cell runs of wire i, sorted by run start.  Returns the count.
__device__ __forceinline__ int neighbour_runs(const CloudGrid& g, const Wire& w,
                                              const int32_t* __restrict__ cell_start,
                                              const int32_t* __restrict__ cell_end,
                                              int32_t* rs, int32_t* re) {
    int ix, iy, iz;
    cell_of(g, w.cx, w.cy, w.cz, ix, iy, iz);
    int nr = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        int z = iz + dz;
        if (z < 0 || z >= g.nz) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            int y = iy + dy;
            if (y < 0 || y >= g.ny) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                int x = ix + dx;
                if (x < 0 || x >= g.nx) continue;
                int64_t lin = g.cell_base + ((int64_t)z * g.ny + y) * g.nx + x;
                int32_t s = cell_start[lin], e = cell_end[lin];
                if (e > s) {
                    int k = nr++;
                    while (k > 0 && rs[k - 1] > s) {  // insertion by run start
                        rs[k] = rs[k - 1];
                        re[k] = re[k - 1];
                        --k;
                    }
                    rs[k] = s;
                    re[k] = e;
                }
            }
        }
    }
    return nr;
}

__global__ void k_count(const Wire* __restrict__ wires, const int32_t* __restrict__ wire_cloud,
                        const CloudGrid* __restrict__ grids, const int32_t* __restrict__ cell_start,
                        const int32_t* __restrict__ cell_end, int64_t n, double dc2,
                        int32_t* __restrict__ cnt, int32_t* __restrict__ cnt_up) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Wire w = wires[i];
        const CloudGrid g = grids[wire_cloud[i]];
        int32_t rs[27], re[27];
        int nr = neighbour_runs(g, w, cell_start, cell_end, rs, re);
        double ci[3] = {w.cx, w.cy, w.cz};
        int32_t c = 0, cu = 0;
        for (int r = 0; r < nr; ++r)
            for (int32_t j = rs[r]; j < re[r]; ++j) {
                double cj[3] = {wires[j].cx, wires[j].cy, wires[j].cz};
                if (j == i || within(ci, cj, dc2)) {
                    ++c;
                    cu += (j > i);
                }
            }
        cnt[i] = c;
        cnt_up[i] = cu;
    }
}

__global__ void k_pattern(const Wire* __restrict__ wires, const int32_t* __restrict__ wire_cloud,
                          const CloudGrid* __restrict__ grids, const int32_t* __restrict__ cell_start,
                          const int32_t* __restrict__ cell_end, int64_t n, double dc2,
                          const int64_t* __restrict__ row_ptr, const int64_t* __restrict__ pair_ptr,
                          int32_t* __restrict__ col_idx, int64_t* __restrict__ diag_pos,
                          Pair* __restrict__ pairs) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const Wire w = wires[i];
        const CloudGrid g = grids[wire_cloud[i]];
        int32_t rs[27], re[27];
        int nr = neighbour_runs(g, w, cell_start, cell_end, rs, re);
        double ci[3] = {w.cx, w.cy, w.cz};
        int64_t pos = row_ptr[i];
        int64_t up = pair_ptr[i];
        for (int r = 0; r < nr; ++r)
            for (int32_t j = rs[r]; j < re[r]; ++j) {
                double cj[3] = {wires[j].cx, wires[j].cy, wires[j].cz};
                if (j == i || within(ci, cj, dc2)) {
                    col_idx[pos] = j;
                    if (j == i) diag_pos[i] = pos;
                    if (j > i) {
                        Pair pr;
                        pr.i = (int32_t)i;
                        pr.j = j;
                        pr.pos_ij = pos;
                        pr.pos_ji = -1;
                        pairs[up++] = pr;
                    }
                    ++pos;
                }
            }
    }
}

__global__ void k_pair_transpose(Pair* __restrict__ pairs, int64_t n_pairs,
                                 const int64_t* __restrict__ row_ptr,
                                 const int32_t* __restrict__ col_idx) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n_pairs;
         e += (int64_t)gridDim.x * blockDim.x) {
        Pair pr = pairs[e];
        int64_t lo = row_ptr[pr.j], hi = row_ptr[pr.j + 1];
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (col_idx[mid] < pr.i) lo = mid + 1; else hi = mid;
        }
        pairs[e].pos_ji = lo;
    }
}

// ------------------------------------------------------------------ host driver

static int64_t cells_cap(int64_t nc) { return std::max<int64_t>(4 * nc, 64); }

struct BuildLayout {
    // persistent (lives with the handle)
    Wire* wires; int32_t* perm; int32_t* iperm; int32_t* wire_cloud;
    int64_t* row_ptr; int32_t* col_idx; int64_t* diag_pos; Pair* pairs; int32_t* status;
    // temporaries
    uint64_t* keys_a; uint64_t* keys_b; int32_t* vals_b;
    int32_t* hist; int32_t* hist_scan; int32_t* sums32; int64_t* sums64;
    int32_t* cnt; int32_t* cnt_up; int64_t* pair_ptr;
    int32_t* cell_start; int32_t* cell_end; double* bbox_part; CloudGrid* grids;
    int64_t* d_off; int32_t* bad;
    size_t bytes;
};

static BuildLayout carve_build(void* ws, size_t ws_bytes, int64_t n, int32_t n_clouds,
                               int64_t max_nnzb) {
    Carve cv(ws, ws_bytes);
    BuildLayout L;
    int64_t max_pairs = std::max<int64_t>((max_nnzb - n) / 2, 1);
    int64_t n_tiles = (n + RS_TILE - 1) / RS_TILE;
    int64_t total_cells = 4 * n + 64 * (int64_t)n_clouds;
    int64_t hist_n = 256 * n_tiles;
    int64_t nsum = (std::max<int64_t>(hist_n, n) + SCAN_BLOCK - 1) / SCAN_BLOCK + 2;
    L.wires = cv.take<Wire>(n);
    L.perm = cv.take<int32_t>(n);
    L.iperm = cv.take<int32_t>(n);
    L.wire_cloud = cv.take<int32_t>(n);
    L.row_ptr = cv.take<int64_t>(n + 1);
    L.col_idx = cv.take<int32_t>(max_nnzb);
    L.diag_pos = cv.take<int64_t>(n);
    L.pairs = cv.take<Pair>(max_pairs);
    L.status = cv.take<int32_t>(64);
    L.keys_a = cv.take<uint64_t>(n);
    L.keys_b = cv.take<uint64_t>(n);
    L.vals_b = cv.take<int32_t>(n);
    L.hist = cv.take<int32_t>(hist_n);
    L.hist_scan = cv.take<int32_t>(hist_n + 1);
    L.sums32 = cv.take<int32_t>(nsum);
    L.sums64 = cv.take<int64_t>(nsum);
    L.cnt = cv.take<int32_t>(n);
    L.cnt_up = cv.take<int32_t>(n);
    L.pair_ptr = cv.take<int64_t>(n + 1);
    L.cell_start = cv.take<int32_t>(total_cells);
    L.cell_end = cv.take<int32_t>(total_cells);
    L.bbox_part = cv.take<double>((int64_t)n_clouds * BBOX_BLOCKS * 6);
    L.grids = cv.take<CloudGrid>(n_clouds);
    L.d_off = cv.take<int64_t>(n_clouds + 1);
    L.bad = cv.take<int32_t>(1);
    L.bytes = cv.off;
    return L;
}

size_t build_workspace_bytes(int64_t n, int32_t n_clouds, int64_t max_nnzb) {
    return carve_build(nullptr, 0, n, n_clouds, max_nnzb).bytes + 256;
}

static int grid1d(int64_t n, int threads = 256, int64_t cap = 65536) {
    int64_t b = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

chaff_status build_cloud(const chaff_params* p, const int64_t* cloud_off, const double* center,
                         const double* tangent, const double* length, const double* radius,
                         void* ws, size_t ws_bytes, int64_t* nnzb_out, hipStream_t st,
                         Cloud** out) {
    const int64_t n = p->n_wires;
    const int32_t nc = p->n_clouds;
    BuildLayout L = carve_build(ws, ws_bytes, n, nc, p->max_nnzb);
    if (L.bytes > ws_bytes)
        return fail(CHAFF_EWORKSPACE, "build workspace too small: need " + std::to_string(L.bytes) +
                                          " bytes, got " + std::to_string(ws_bytes));

    std::vector<CloudGrid> grids(nc);
    for (int c = 0; c < nc; ++c) {
        grids[c] = CloudGrid{};
        grids[c].w0 = cloud_off[c];
        grids[c].w1 = cloud_off[c + 1];
    }
    std::vector<int64_t> offv(cloud_off, cloud_off + nc + 1);
    CHAFF_HIP(hipMemcpyAsync(L.d_off, offv.data(), (nc + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, L.bad, (int64_t)1, 0);
    CHAFF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bbox, dim3(BBOX_BLOCKS, nc), dim3(256), 0, st, center, tangent, length, radius,
                       (const int64_t*)L.d_off, L.bbox_part, L.bad, (int)p->n_seg);
    CHAFF_LAUNCH_CHECK();
    std::vector<double> part((size_t)nc * BBOX_BLOCKS * 6);
    int32_t bad = 0;
    CHAFF_HIP(hipMemcpyAsync(part.data(), L.bbox_part, part.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipMemcpyAsync(&bad, L.bad, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipStreamSynchronize(st));
    if (bad)
        return fail(CHAFF_EINVAL, std::to_string(bad) +
                                      " wires have a non-finite centre, a tangent that is not unit "
                                      "length (|t|^2 off by > 1e-10), length <= 0 or a radius outside "
                                      "(0, length/n_seg)");

    // --- cell grid per cloud: side strictly above d_c, bounded table size
    int64_t cell_base = 0;
    int dim_bits = 0;
    for (int c = 0; c < nc; ++c) {
        double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int b = 0; b < BBOX_BLOCKS; ++b) {
            const double* q = &part[((size_t)c * BBOX_BLOCKS + b) * 6];
            for (int d = 0; d < 3; ++d) {
                mn[d] = std::min(mn[d], q[d]);
                mx[d] = std::max(mx[d], q[3 + d]);
            }
        }
        CloudGrid& g = grids[c];
        int64_t ncw = g.w1 - g.w0;
        if (ncw == 0) {
            mn[0] = mn[1] = mn[2] = 0;
            mx[0] = mx[1] = mx[2] = 0;
        }
        g.ox = mn[0]; g.oy = mn[1]; g.oz = mn[2];
        double ext = std::max({mx[0] - mn[0], mx[1] - mn[1], mx[2] - mn[2], 0.0});
        g.nx = g.ny = g.nz = 1;
        g.inv_h = 0.0;
        double dc = p->d_c;
        if (std::isfinite(dc) && dc * (1.0 + 1e-9) < ext) {
            double h = std::max({dc * (1.0 + 1e-9), ext / 65000.0, 1e-30});
            const int64_t cap = cells_cap(ncw);
            for (;;) {
                double ax = (mx[0] - mn[0]) / h, ay = (mx[1] - mn[1]) / h, az = (mx[2] - mn[2]) / h;
                double cells = (std::floor(ax) + 1) * (std::floor(ay) + 1) * (std::floor(az) + 1);
                if (cells <= (double)cap && ax < 65000 && ay < 65000 && az < 65000) {
                    g.nx = (int)std::floor(ax) + 1;
                    g.ny = (int)std::floor(ay) + 1;
                    g.nz = (int)std::floor(az) + 1;
                    break;
                }
                h *= 1.25;
            }
            g.inv_h = 1.0 / h;
        }
        g.cell_base = cell_base;
        cell_base += (int64_t)g.nx * g.ny * g.nz;
        int mdim = std::max({g.nx, g.ny, g.nz});
        int bits = 0;
        while ((1 << bits) < mdim) ++bits;
        dim_bits = std::max(dim_bits, bits);
    }
    const int64_t total_cells = cell_base;
    if (total_cells > 4 * n + 64 * (int64_t)nc) return fail(CHAFF_EINVAL, "internal: cell table overflow");
    int cloud_bits = 0;
    while ((1 << cloud_bits) < nc) ++cloud_bits;
    const int key_bits = 3 * dim_bits + cloud_bits;
    CHAFF_HIP(hipMemcpyAsync(L.grids, grids.data(), nc * sizeof(CloudGrid), hipMemcpyHostToDevice, st));

    // --- keys and a stable LSD radix sort (perm = caller index in sorted order)
    int64_t maxc = 1;
    for (int c = 0; c < nc; ++c) maxc = std::max<int64_t>(maxc, grids[c].w1 - grids[c].w0);
    hipLaunchKernelGGL(k_keys, dim3(grid1d(maxc, 256, 4096), nc), dim3(256), 0, st, center,
                       (const CloudGrid*)L.grids, dim_bits, L.keys_a, L.perm);
    CHAFF_LAUNCH_CHECK();
    const int n_tiles = (int)((n + RS_TILE - 1) / RS_TILE);
    uint64_t* kin = L.keys_a; int32_t* vin = L.perm;
    uint64_t* kout = L.keys_b; int32_t* vout = L.vals_b;
    const int passes = (key_bits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
        ProfScope prof_sort("nbr_sort_pass", st);
        hipLaunchKernelGGL(k_rs_hist, dim3(n_tiles), dim3(RS_THREADS), 0, st, (const uint64_t*)kin, n,
                           8 * ps, L.hist, n_tiles);
        CHAFF_LAUNCH_CHECK();
        chaff_status s = exclusive_scan<int32_t, int32_t>(L.hist, (int64_t)256 * n_tiles, L.hist_scan,
                                                          L.sums32, st);
        if (s != CHAFF_OK) return s;
        hipLaunchKernelGGL(k_rs_scatter, dim3(n_tiles), dim3(RS_THREADS), 0, st, (const uint64_t*)kin,
                           (const int32_t*)vin, kout, vout, n, 8 * ps, (const int32_t*)L.hist_scan, n_tiles);
        CHAFF_LAUNCH_CHECK();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    if (vin != L.perm) {  // odd pass count: bring the result home
        CHAFF_HIP(hipMemcpyAsync(L.perm, vin, n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
        CHAFF_HIP(hipMemcpyAsync(L.keys_a, kin, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
    }
    const uint64_t* keys = L.keys_a;

    // --- internal geometry and cell tables
    hipLaunchKernelGGL(k_gather, dim3(grid1d(n)), dim3(256), 0, st, center, tangent, length, radius,
                       (const int32_t*)L.perm, (const CloudGrid*)L.grids, nc, n, L.wires, L.iperm,
                       L.wire_cloud);
    CHAFF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1d(total_cells)), dim3(256), 0, st, L.cell_start, total_cells, 0);
    CHAFF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1d(total_cells)), dim3(256), 0, st, L.cell_end, total_cells, 0);
    CHAFF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cells, dim3(grid1d(n)), dim3(256), 0, st, (const Wire*)L.wires,
                       (const int32_t*)L.wire_cloud, keys, (const CloudGrid*)L.grids, n, L.cell_start,
                       L.cell_end);
    CHAFF_LAUNCH_CHECK();

    // --- pass 1: counts, scans, read-back
    const double dc2 = std::isfinite(p->d_c) ? p->d_c * p->d_c : INFINITY;
    {
        ProfScope pc("nbr_count", st);
        hipLaunchKernelGGL(k_count, dim3(grid1d(n, 128)), dim3(128), 0, st, (const Wire*)L.wires,
                           (const int32_t*)L.wire_cloud, (const CloudGrid*)L.grids,
                           (const int32_t*)L.cell_start, (const int32_t*)L.cell_end, n, dc2, L.cnt, L.cnt_up);
    }
    CHAFF_LAUNCH_CHECK();
    chaff_status s1 = exclusive_scan<int32_t, int64_t>(L.cnt, n, L.row_ptr, L.sums64, st);
    if (s1 != CHAFF_OK) return s1;
    s1 = exclusive_scan<int32_t, int64_t>(L.cnt_up, n, L.pair_ptr, L.sums64, st);
    if (s1 != CHAFF_OK) return s1;
    int64_t tot[2] = {0, 0};
    CHAFF_HIP(hipMemcpyAsync(&tot[0], L.row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipMemcpyAsync(&tot[1], L.pair_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    CHAFF_HIP(hipStreamSynchronize(st));
    const int64_t nnzb = tot[0], n_pairs = tot[1];
    *nnzb_out = nnzb;
    if (nnzb > p->max_nnzb || n_pairs > std::max<int64_t>((p->max_nnzb - n) / 2, 1))
        return fail(CHAFF_EWORKSPACE, "pattern needs " + std::to_string(nnzb) +
                                          " blocks, capacity max_nnzb = " + std::to_string(p->max_nnzb));
    if (nnzb != n + 2 * n_pairs) return fail(CHAFF_EINVAL, "internal: asymmetric near set");

    // --- pass 2: column indices, diagonal positions, unique pairs
    {
        ProfScope pp("nbr_pattern", st);
        hipLaunchKernelGGL(k_pattern, dim3(grid1d(n, 128)), dim3(128), 0, st, (const Wire*)L.wires,
                           (const int32_t*)L.wire_cloud, (const CloudGrid*)L.grids,
                           (const int32_t*)L.cell_start, (const int32_t*)L.cell_end, n, dc2,
                           (const int64_t*)L.row_ptr, (const int64_t*)L.pair_ptr, L.col_idx, L.diag_pos,
                           L.pairs);
    }
    CHAFF_LAUNCH_CHECK();
    if (n_pairs > 0) {
        hipLaunchKernelGGL(k_pair_transpose, dim3(grid1d(n_pairs)), dim3(256), 0, st, L.pairs, n_pairs,
                           (const int64_t*)L.row_ptr, (const int32_t*)L.col_idx);
        CHAFF_LAUNCH_CHECK();
    }

    Cloud* c = new Cloud();
    c->n = n;
    c->nnzb = nnzb;
    c->n_pairs = n_pairs;
    c->max_nnzb = p->max_nnzb;
    c->n_clouds = nc;
    c->wavelength = p->wavelength;
    c->d_c = p->d_c;
    c->q_mutual = p->quad_mutual;
    c->q_self = p->quad_self;
    c->nseg = p->n_seg;
    c->cloud_off = offv;
    c->wires = L.wires;
    c->perm = L.perm;
    c->iperm = L.iperm;
    c->wire_cloud = L.wire_cloud;
    c->row_ptr = L.row_ptr;
    c->col_idx = L.col_idx;
    c->diag_pos = L.diag_pos;
    c->pairs = L.pairs;
    c->d_status = L.status;
    gauss_legendre01(c->q_mutual, c->xq_m, c->wq_m);
    gauss_legendre01(c->q_self, c->xq_s, c->wq_s);
    *out = c;
    return CHAFF_OK;
}

}  // namespace chaff
