// Far-field reduction: monostatic and bistatic RCS (Sec. III).
//
// S(r_hat, e) = sum_p (t_p . e) exp(+j k r_hat . c_p) D_p sinc^2(b D_p / 2)
//               * sum_q x_{p,q} exp(+j b s_q),     b = k r_hat . t_p,
// the closed-form triangle transform of every rooftop; sigma = |S|^2/(4 pi).
// Everything is FP64 (the phase k r_hat . c_p reaches hundreds of radians).
//
//  * monostatic: direction m pairs with RHS m; blocks reduce fixed wire
//    chunks of one cloud, lanes split between RHS columns and wire slots, the
//    slots folded with wavefront shuffles and the waves through LDS; a second
//    pass sums the chunks of each cloud in order (no atomics, bit-reproducible);
//  * bistatic: one thread per direction, the chunk's wires and currents
//    staged in LDS, partial sums per chunk, same second pass.
#include "common.hpp"
#include "prof.hpp"

#include <algorithm>
#include <mutex>

namespace chaff {

constexpr double PI_F = 3.14159265358979323846;
// wires per chunk: 256 for 7 unknowns per wire, 64 for 19 (the bistatic
// kernel stages a chunk's currents in LDS)
constexpr int ff_chunk(int nb) { return nb <= 7 ? 256 : 64; }

__device__ __forceinline__ double sinc_ff(double x) {
    return fabs(x) < 1e-4 ? 1.0 - x * x / 6.0 : sin(x) / x;
}

// one wire's contribution for direction (rx,ry,rz), polarisation (ex,ey,ez)
template <int NBW>
__device__ __forceinline__ c128 wire_term(const Wire& w, const c128* __restrict__ x, int64_t xstride, double k,
                                          double rx, double ry, double rz, double ex, double ey, double ez) {
    const double tp = w.tx * ex + w.ty * ey + w.tz * ez;
    const double b = k * (rx * w.tx + ry * w.ty + rz * w.tz);
    const double ph0 = k * (rx * w.cx + ry * w.cy + rz * w.cz);
    const double D = w.len / (NBW + 1);
    const double sc = sinc_ff(0.5 * b * D);
    const double env = tp * D * sc * sc;
    // exp(j b s_q), s_q = -L/2 + (q+1) D, by recurrence in q
    double s1, c1, sd, cd;
    sincos(ph0 + b * (-0.5 * w.len + D), &s1, &c1);
    sincos(b * D, &sd, &cd);
    c128 ph = {c1, s1};
    const c128 step = {cd, sd};
    c128 acc = {0, 0};
    for (int q = 0; q < NBW; ++q) {
        cfma(acc, ph, x[q * xstride]);
        ph = cmul(ph, step);
    }
    return cscale(acc, env);
}

// partial[chunk][r] for monostatic pairs (dir r, rhs r); X caller order.
// A wave is RT RHS columns x (64 / RT) wire slots: lane (g, c) = (lane / RT,
// lane % RT) sums the terms of wires w0 + (4 wv + g) + 256/RT * k, so a wire
// row of RT columns is one contiguous load for the RT lanes of a slot.  The
// slots are then folded with wavefront shuffles (xor over the slot bits) and
// the four waves combined in wave order through LDS: a fixed summation order
// (bit-reproducible, no atomics).  RT is the smallest power of two >= R
// (at most 64), so few RHS columns do not leave lanes idle.
template <int RT, int NBW>
__global__ __launch_bounds__(256) void k_mono(const Wire* __restrict__ wires, const int32_t* __restrict__ perm,
                                              const int64_t* __restrict__ chunk_w0, int n_chunks, int64_t R,
                                              const c128* __restrict__ X, const double* __restrict__ dir,
                                              const double* __restrict__ pol, double k, c128* __restrict__ part) {
    constexpr int G = 64 / RT;   // wire slots per wave
    __shared__ c128 red[4][RT];
    const int ch = blockIdx.x;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane / RT, c = lane % RT;
    const int64_t r = (int64_t)blockIdx.y * RT + c;
    const int64_t w0 = chunk_w0[ch], w1 = chunk_w0[ch + 1];
    c128 acc = {0, 0};
    if (r < R) {
        const double rx = dir[3 * r], ry = dir[3 * r + 1], rz = dir[3 * r + 2];
        const double ex = pol[3 * r], ey = pol[3 * r + 1], ez = pol[3 * r + 2];
        for (int64_t i = w0 + wv * G + g; i < w1; i += 4 * G) {
            const Wire wr = wires[i];
            const c128* xp = X + (int64_t)perm[i] * NBW * R + r;
            acc = cadd(acc, wire_term<NBW>(wr, xp, R, k, rx, ry, rz, ex, ey, ez));
        }
    }
#pragma unroll
    for (int off = RT; off < 64; off <<= 1) {
        acc.re += __shfl_xor(acc.re, off, 64);
        acc.im += __shfl_xor(acc.im, off, 64);
    }
    if (g == 0) red[wv][c] = acc;
    __syncthreads();
    if (wv == 0 && g == 0 && r < R) {
        c128 t = red[0][c];
        for (int q = 1; q < 4; ++q) t = cadd(t, red[q][c]);
        part[(int64_t)ch * R + r] = t;
    }
}

template <int NBW>
static void launch_mono(dim3 grid_x, int64_t R, hipStream_t st, const Wire* wires, const int32_t* perm,
                        const int64_t* w0, int nch, const c128* X, const double* dir, const double* pol, double k,
                        c128* part) {
    const int rt = R >= 64 ? 64 : R > 16 ? 32 : R > 8 ? 16 : R > 4 ? 8 : R > 2 ? 4 : R > 1 ? 2 : 1;
    const dim3 grid(grid_x.x, (unsigned)((R + rt - 1) / rt));
    switch (rt) {
#define CHAFF_MONO(T) \
    case T: hipLaunchKernelGGL((k_mono<T, NBW>), grid, dim3(256), 0, st, wires, perm, w0, nch, R, X, dir, pol, k, part); break;
        CHAFF_MONO(1) CHAFF_MONO(2) CHAFF_MONO(4) CHAFF_MONO(8) CHAFF_MONO(16) CHAFF_MONO(32) CHAFF_MONO(64)
#undef CHAFF_MONO
    }
}

// partial[chunk][r][m] for every (rhs r, direction m)
template <int NBW>
__global__ __launch_bounds__(256) void k_bistatic(const Wire* __restrict__ wires, const int32_t* __restrict__ perm,
                                                  const int64_t* __restrict__ chunk_w0, int64_t R, int64_t M,
                                                  const c128* __restrict__ X, const double* __restrict__ dir,
                                                  const double* __restrict__ pol, double k, c128* __restrict__ part) {
    constexpr int CH = ff_chunk(NBW);
    __shared__ Wire sw[CH];
    __shared__ c128 sx[CH * NBW];
    const int ch = blockIdx.y;
    const int64_t r = blockIdx.z;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w0 = chunk_w0[ch], w1 = chunk_w0[ch + 1];
    const int nw = (int)(w1 - w0);
    for (int t = threadIdx.x; t < nw; t += blockDim.x) {
        sw[t] = wires[w0 + t];
        const int64_t p = perm[w0 + t];
        for (int q = 0; q < NBW; ++q) sx[t * NBW + q] = X[(p * NBW + q) * R + r];
    }
    __syncthreads();
    if (m >= M) return;
    const double rx = dir[3 * m], ry = dir[3 * m + 1], rz = dir[3 * m + 2];
    const double ex = pol[3 * m], ey = pol[3 * m + 1], ez = pol[3 * m + 2];
    c128 acc = {0, 0};
    for (int t = 0; t < nw; ++t) acc = cadd(acc, wire_term<NBW>(sw[t], &sx[t * NBW], 1, k, rx, ry, rz, ex, ey, ez));
    part[((int64_t)ch * R + r) * M + m] = acc;
}

// sigma[cloud][j] = |sum over the cloud's chunks of part[chunk][j]|^2 / (4 pi), j < J
__global__ void k_ff_finish(const c128* __restrict__ part, const int32_t* __restrict__ cloud_chunk_off,
                            int n_clouds, int64_t J, double* __restrict__ sigma) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_clouds * J) return;
    const int c = (int)(t / J);
    const int64_t j = t - (int64_t)c * J;
    c128 acc = {0, 0};
    for (int ch = cloud_chunk_off[c]; ch < cloud_chunk_off[c + 1]; ++ch) acc = cadd(acc, part[(int64_t)ch * J + j]);
    sigma[t] = (acc.re * acc.re + acc.im * acc.im) / (4.0 * PI_F);
}

static void ff_chunks(const Cloud* c, std::vector<int64_t>& w0, std::vector<int32_t>& coff) {
    w0.clear();
    coff.assign(c->n_clouds + 1, 0);
    for (int k = 0; k < c->n_clouds; ++k) {
        coff[k] = (int32_t)w0.size();
        for (int64_t a = c->cloud_off[k]; a < c->cloud_off[k + 1]; a += ff_chunk(c->nseg - 1)) w0.push_back(a);
    }
    coff[c->n_clouds] = (int32_t)w0.size();
}

size_t rcs_workspace_bytes(const Cloud* c, int64_t R, int64_t M, int32_t mono) {
    std::vector<int64_t> w0;
    std::vector<int32_t> coff;
    ff_chunks(c, w0, coff);
    const int64_t nch = (int64_t)w0.size();
    const int64_t J = mono ? R : R * M;
    size_t b = align_up((nch + 1) * sizeof(int64_t), 256) + align_up((c->n_clouds + 1) * sizeof(int32_t), 256) +
               align_up((size_t)std::max<int64_t>(nch, 1) * J * sizeof(c128), 256);
    return b + 256;
}

chaff_status rcs(Cloud* c, const void* Xv, int64_t R, const double* dir, const double* pol, int64_t M, int32_t mono,
                 double* sigma, void* ws, size_t ws_bytes, hipStream_t st) {
    std::vector<int64_t> w0;
    std::vector<int32_t> coff;
    ff_chunks(c, w0, coff);
    const int nch = (int)w0.size();
    const int64_t J = mono ? R : R * M;
    Carve cv(ws, ws_bytes);
    int64_t* d_w0 = cv.take<int64_t>(nch + 1);
    int32_t* d_coff = cv.take<int32_t>(c->n_clouds + 1);
    c128* part = cv.take<c128>((size_t)std::max(nch, 1) * J);
    if (!cv.ok()) return fail(CHAFF_EWORKSPACE, "rcs workspace too small");
    // chunk i covers wires [bounds[i], bounds[i+1]); chunks start at cloud
    // boundaries, so the next chunk's start is always this chunk's end
    std::vector<int64_t> bounds(w0);
    bounds.push_back(c->n);
    CHAFF_HIP(hipMemcpyAsync(d_w0, bounds.data(), bounds.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    CHAFF_HIP(hipMemcpyAsync(d_coff, coff.data(), coff.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    const double k = 2.0 * PI_F / c->wavelength;
    const c128* X = static_cast<const c128*>(Xv);
    if (nch > 0) {
        // monostatic: X read once + wire records; bistatic: 55 flops per wire and direction
        ProfScope ps(mono ? "rcs_mono" : "rcs_bistatic", st,
                     mono ? 16.0 * (c->nseg - 1) * (double)c->n * R + 64.0 * c->n
                          : 55.0 * (double)c->n * R * M, !mono);
        if (mono) {
            if (c->nseg == NSEG)
                launch_mono<NSEG - 1>(dim3(nch), R, st, (const Wire*)c->wires, (const int32_t*)c->perm,
                                      (const int64_t*)d_w0, nch, X, dir, pol, k, part);
            else
                launch_mono<NSEG_PAPER - 1>(dim3(nch), R, st, (const Wire*)c->wires, (const int32_t*)c->perm,
                                            (const int64_t*)d_w0, nch, X, dir, pol, k, part);
        } else {
            dim3 grid((unsigned)((M + 255) / 256), nch, (unsigned)R);
            if (c->nseg == NSEG)
                hipLaunchKernelGGL(k_bistatic<NSEG - 1>, grid, dim3(256), 0, st, (const Wire*)c->wires,
                                   (const int32_t*)c->perm, (const int64_t*)d_w0, R, M, X, dir, pol, k, part);
            else
                hipLaunchKernelGGL(k_bistatic<NSEG_PAPER - 1>, grid, dim3(256), 0, st, (const Wire*)c->wires,
                                   (const int32_t*)c->perm, (const int64_t*)d_w0, R, M, X, dir, pol, k, part);
        }
        CHAFF_LAUNCH_CHECK();
    }
    const int64_t tot = (int64_t)c->n_clouds * J;
    hipLaunchKernelGGL(k_ff_finish, dim3((unsigned)std::max<int64_t>(1, (tot + 255) / 256)), dim3(256), 0, st,
                       (const c128*)part, (const int32_t*)d_coff, c->n_clouds, J, sigma);
    CHAFF_LAUNCH_CHECK();
    CHAFF_HIP(hipStreamSynchronize(st));  // host staging vectors go out of scope
    return CHAFF_OK;
}

// ------------------------------------------------------------------ far field without a workspace
// The scratch of chaff_rcs (chunk bounds, cloud chunk offsets, per-chunk
// partial sums) in a fixed device array of the library, one copy per GPU.  The
// array's name is only a host-side stand-in: its device address on the current
// GPU is looked up once per device with hipGetSymbolAddress and used for every
// kernel argument and copy.
static __device__ __align__(256) unsigned char scratch[CHAFF_RCS_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static chaff_status scratch_address(void** out) {
    int dev = -1;
    CHAFF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(CHAFF_EINVAL, "device index out of range for the fixed scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        CHAFF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(CHAFF_EHIP, "hipGetSymbolAddress returned no address for the fixed scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CHAFF_OK;
}

chaff_status rcs_noalloc(Cloud* c, const void* X, int64_t R, const double* dir, const double* pol, int64_t M,
                         int32_t mono, double* sigma, hipStream_t st) {
    const size_t need = rcs_workspace_bytes(c, R, M, mono);
    if (need > (size_t)CHAFF_RCS_SCRATCH_BYTES)
        return fail(CHAFF_EWORKSPACE, "rcs scratch of " + std::to_string(need) + " bytes exceeds the fixed " +
                                          std::to_string((size_t)CHAFF_RCS_SCRATCH_BYTES) + " bytes");
    void* ws = nullptr;
    chaff_status e = scratch_address(&ws);
    if (e != CHAFF_OK) return e;
    return rcs(c, X, R, dir, pol, M, mono, sigma, ws, (size_t)CHAFF_RCS_SCRATCH_BYTES, st);
}

}  // namespace chaff
