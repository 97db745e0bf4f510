// Cluster block-Jacobi preconditioner: definitions shared by its kernels and the
// Krylov solver.
#pragma once

#include "common.hpp"

namespace chaff {

constexpr int CLW = 8;                 // wires per cluster
constexpr int CLR = CLW * NB;          // rows (and columns) of a cluster block: 56
constexpr int CLR2 = CLR * CLR;        // complex entries per cluster block

struct ClusterEntry {   // one cluster: wires [w0, w0 + nw) of the internal order
    int32_t w0, nw;
};
static_assert(sizeof(ClusterEntry) == 8, "ClusterEntry is 8 bytes");

// Clusters of the cloud: runs of CLW consecutive wires of one cloud.
int64_t cluster_count(const Cloud* c);
// Bytes of the caller's preconditioner buffer: the cluster table (padded to
// 256 bytes), then n_clusters blocks of CLR x CLR complex (prec).
size_t cluster_table_bytes(int64_t n_cl);
size_t cluster_buffer_bytes(const Cloud* c, chaff_prec prec);

// Host check that M's first and last table entries are those of this cloud
// (guards against passing another buffer as the cluster preconditioner).
chaff_status cluster_check_table(const Cloud* c, const void* M, hipStream_t st);

// Y = M X (or Y += M X with accumulate) on the internal order, [rows][s];
// x64 / y64 select complex double for X / Y (else the complex type of prec).
chaff_status cluster_apply_launch(const Cloud* c, chaff_prec prec, const void* M, const void* X, bool x64, void* Y,
                                  bool y64, bool accumulate, int64_t s, hipStream_t st, const char* prof_name);

// ------------------------------------------------------------------ neighbourhood inverse
// The block-diagonal preconditioner of Sec. II-B centred on every wire: wire
// p's neighbourhood is p and its nearest near-set neighbours (at most `size`
// wires); p's row of M is its row block of the inverse of the neighbourhood's
// submatrix of Z, and M_pq = (W_p[p,q] + W_q[q,p]^T) / 2 keeps M complex
// symmetric.  M is stored on Z's block pattern.
constexpr int NBH_MAX = 8;                         // wires per neighbourhood at most
constexpr size_t NBH_HEADER = 256;                 // bytes of the buffer header
constexpr int64_t NBH_MAGIC = 0x3148424e46464843ll;   // "CHFFNBH1"
struct NbhdHeader {
    int64_t magic, n, nnzb;
    int32_t size, prec;
    int32_t raw, pad;    // raw = 1: unsymmetrised rows (training targets), refused by the solver
};
// Buffer: header (256 B), [N][size] int32 neighbourhood table (internal
// indices, slot 0 the wire itself, -1 unused) padded to 256 B, then
// [nnzb][NB][NB] complex (prec) in Z's block order.
size_t nbhd_table_bytes(int64_t n, int size);
size_t nbhd_buffer_bytes(const Cloud* c, chaff_prec prec, int size);
chaff_status nbhd_precond(Cloud* c, chaff_prec prec, int size, const void* Z, void* M, bool raw, hipStream_t st);
// Steps shared with the learned form: the header, zeroed blocks and the
// neighbourhood table; the symmetrisation of raw rows in place.
chaff_status nbhd_begin(Cloud* c, chaff_prec prec, int size, bool raw, void* M, hipStream_t st);
chaff_status nbhd_symmetrise(Cloud* c, chaff_prec prec, void* vals, hipStream_t st);
// Reads M's header (host-synchronising) and checks it against the cloud.
chaff_status nbhd_header(const Cloud* c, const void* M, NbhdHeader* h, hipStream_t st);
// Host check of M's header against the cloud (host-synchronising); returns
// the neighbourhood size through *size.
chaff_status nbhd_check(const Cloud* c, chaff_prec prec, const void* M, int* size, hipStream_t st);
inline size_t nbhd_blocks_offset(int64_t n, int size) { return NBH_HEADER + nbhd_table_bytes(n, size); }

// Rows of one cluster product y = M x for the calling lane: rows
// rho = rsub * RPT + j (j < RPT) of the 56 x 56 block, column col of the
// LDS tile xs [56][ST].  The block comes from LDS (ms, row-major, when it was
// staged there) or straight from memory (mb).  With FULL (NSUB * RPT == 56)
// every row exists and no guard is emitted; with 64-column tiles the rows are
// wave-uniform, so every read of the block is a broadcast.
// CW adjacent columns per lane (col, col + 1, ...): each value read from the
// block then serves CW columns.
template <typename R, typename CZ, int ST, int RPT, bool FULL, bool STAGED, int CW = 1>
__device__ __forceinline__ void cluster_rows(const CZ* __restrict__ ms, const CZ* __restrict__ mb,
                                             const cplx<R>* __restrict__ xs, int col, int rsub,
                                             cplx<R> (&acc)[RPT * CW]) {
#pragma unroll
    for (int j = 0; j < RPT * CW; ++j) acc[j] = cplx<R>{0, 0};
#pragma unroll 2
    for (int k = 0; k < CLR; k += 2) {
        cplx<R> x0[CW], x1[CW];
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) {
            x0[cc] = xs[k * ST + col + cc];
            x1[cc] = xs[(k + 1) * ST + col + cc];
        }
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int rho = rsub * RPT + j;
            if (FULL || rho < CLR) {
                const CZ* row = (STAGED ? ms : mb) + rho * CLR + k;
                const cplx<R> m0 = ccast<cplx<R>>(row[0]), m1 = ccast<cplx<R>>(row[1]);
#pragma unroll
                for (int cc = 0; cc < CW; ++cc) {
                    cfma(acc[j * CW + cc], m0, x0[cc]);
                    cfma(acc[j * CW + cc], m1, x1[cc]);
                }
            }
        }
    }
}

// Cooperative copy of one cluster block into LDS with 16-byte accesses.
template <typename CZ, int NT>
__device__ __forceinline__ void stage_block(CZ* __restrict__ ms, const CZ* __restrict__ mb) {
    static_assert((CLR2 * sizeof(CZ)) % 16 == 0, "block is a whole number of 16-byte words");
    const float4* src = reinterpret_cast<const float4*>(mb);
    float4* dst = reinterpret_cast<float4*>(ms);
    constexpr int WORDS = CLR2 * (int)sizeof(CZ) / 16;
    for (int e = threadIdx.x; e < WORDS; e += NT) dst[e] = src[e];
}

}  // namespace chaff
