// Internal definitions shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/chaff.h"

namespace chaff {

// Segments per wire of the 8-segment kernels (neighbour features of the learned
// guess, cluster preconditioner); the fill, products, solvers and far field
// also run the paper's 20 segments (Cloud::nseg).
constexpr int NSEG = 8;      // segments per wire
constexpr int NB = 7;        // rooftop unknowns per wire
constexpr int NB2 = NB * NB; // complex entries per block
constexpr int NSEG_PAPER = 20;  // the discretisation of the paper's own runs (19 unknowns per wire)
constexpr int MAXQ = 8;      // largest Gauss-Legendre order supported

// ------------------------------------------------------------------ complex
template <typename R>
struct cplx {
    R re, im;
};
using c64 = cplx<float>;
using c128 = cplx<double>;

template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmk(R a, R b) { return {a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a += b*c
template <typename R>
__host__ __device__ __forceinline__ void cfma(cplx<R>& a, cplx<R> b, cplx<R> c) {
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(-b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(b.im, c.re, a.im);
}
// a += conj(b)*c
template <typename R>
__host__ __device__ __forceinline__ void cfma_conj(cplx<R>& a, cplx<R> b, cplx<R> c) {
    a.re = fma(b.re, c.re, a.re);
    a.re = fma(b.im, c.im, a.re);
    a.im = fma(b.re, c.im, a.im);
    a.im = fma(-b.im, c.re, a.im);
}
template <typename R>
__host__ __device__ __forceinline__ cplx<R> cscale(cplx<R> a, R s) { return {a.re * s, a.im * s}; }

template <typename T>
struct real_of;
template <>
struct real_of<c64> { using type = float; };
template <>
struct real_of<c128> { using type = double; };

template <typename To, typename From>
__host__ __device__ __forceinline__ To ccast(From a) {
    using R = typename real_of<To>::type;
    return To{static_cast<R>(a.re), static_cast<R>(a.im)};
}

// ------------------------------------------------------------------ geometry
// One wire in internal order.  FP64 so that pair separations are formed
// before any rounding to FP32.
struct Wire {
    double cx, cy, cz;   // centre
    double tx, ty, tz;   // unit tangent
    double len;          // length
    double rad;          // radius
};
static_assert(sizeof(Wire) == 64, "Wire is 64 bytes");

struct Pair {            // unique off-diagonal pair i < j (internal indices)
    int32_t i, j;
    int64_t pos_ij;      // block index of (i, j)
    int64_t pos_ji;      // block index of (j, i)
};
static_assert(sizeof(Pair) == 24, "Pair is 24 bytes");

struct CloudGrid {       // per-cloud cell grid for the neighbour search
    double ox, oy, oz;   // origin (cloud minimum corner)
    double inv_h;        // 1 / cell side (0 for the single-cell dense case)
    int32_t nx, ny, nz;  // cells per axis (each <= 65535)
    int32_t pad;
    int64_t cell_base;   // offset of this cloud's cells in the dense tables
    int64_t w0, w1;      // wire range [w0, w1)
};

// ------------------------------------------------------------------ handle
struct Cloud {
    int64_t n = 0, nnzb = 0, n_pairs = 0, max_nnzb = 0;
    int32_t n_clouds = 1;
    double wavelength = 0, d_c = 0;
    int32_t q_mutual = 4, q_self = 8;
    int32_t nseg = NSEG;                 // segments per wire: 8 or 20
    std::vector<int64_t> cloud_off;      // host copy
    // device arrays (inside the caller's build workspace)
    Wire* wires = nullptr;               // [N] internal order
    int32_t* perm = nullptr;             // [N] internal -> caller
    int32_t* iperm = nullptr;            // [N] caller -> internal
    int32_t* wire_cloud = nullptr;       // [N] cloud of internal wire
    int64_t* row_ptr = nullptr;          // [N+1]
    int32_t* col_idx = nullptr;          // [max_nnzb]
    int64_t* diag_pos = nullptr;         // [N]
    Pair* pairs = nullptr;               // [max_pairs]
    int32_t* d_status = nullptr;         // small device status words
    // gauss nodes (host, FP64)
    double xq_m[MAXQ], wq_m[MAXQ], xq_s[MAXQ], wq_s[MAXQ];
};

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
chaff_status fail(chaff_status st, const std::string& msg);

#define CHAFF_HIP(call)                                                              \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::chaff::fail(CHAFF_EHIP, std::string(#call) + ": " +             \
                                 hipGetErrorString(e_));                             \
    } while (0)

#define CHAFF_LAUNCH_CHECK()                                                         \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess)                                                        \
            return ::chaff::fail(CHAFF_EHIP, std::string("kernel launch: ") +        \
                                 hipGetErrorString(e_) + " at " + __FILE__ + ":" +   \
                                 std::to_string(__LINE__));                          \
    } while (0)

// Gauss-Legendre nodes/weights on [0,1] (Newton on Legendre polynomials).
void gauss_legendre01(int q, double* x, double* w);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over a caller workspace.
struct Carve {
    char* base;
    size_t off = 0, cap;
    Carve(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        off = align_up(off, 256);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    bool ok() const { return off <= cap; }
};

}  // namespace chaff
