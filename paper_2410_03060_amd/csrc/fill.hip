// Galerkin impedance fill (eqs. 5-8) on the S-NFC pattern.
//
//  * Mutual blocks: one wave64 per unique wire pair (i < j).  Lane
//    (alpha, beta) = (lane/8, lane%8) owns one of the 8 x 8 segment pairs and
//    runs the Q x Q Gauss samples of G for it, accumulating the four
//    first-order moments of the rooftop halves.  The pair separation and the
//    segment offsets are formed in FP64 and rounded once; the samples run in
//    the block precision R.  The 7 x 7 block is assembled with cross-lane
//    permutes (each output needs the four segment pairs its two rooftops
//    overlap) and stored twice: Z_ij and Z_ji = Z_ij^T.
//  * Self blocks: eight wires per wave64.  They are Toeplitz in the segment
//    offset d = alpha - beta, so lane (wire g, offset d) runs the samples of
//    one offset; for d <= 1 the static part 1/(4 pi R) is added in closed
//    form (FP64 iterated antiderivatives) and only (exp(-jkR) - 1)/(4 pi R)
//    is sampled.  A separate pass inverts the blocks for the block-diagonal
//    preconditioner, one lane per wire (Gauss-Jordan, partial pivoting).
//  * 20 segments (the paper's own discretisation): one wave per pair or wire,
//    lanes looping over the segment pairs or offsets (k_mutual_w, k_self_w).
#include "common.hpp"
#include "prof.hpp"

namespace chaff {

constexpr double PI = 3.14159265358979323846;

struct FillParams {
    double k;            // wavenumber
    double inv_lambda;   // 1 / wavelength
    int32_t q;           // Gauss order
    int32_t pad;
    double xq[MAXQ];     // nodes on [0,1]
    double wq[MAXQ];     // weights
};

// exp(-j 2 pi rev) split into (cos, -sin) with the phase in revolutions.
__device__ __forceinline__ void phase_cs(float rev, float& c, float& s) {
    float f = __builtin_amdgcn_fractf(rev);
    s = __builtin_amdgcn_sinf(f);   // sin(2 pi f)
    c = __builtin_amdgcn_cosf(f);   // cos(2 pi f)
}
__device__ __forceinline__ void phase_cs(double rev, double& c, double& s) {
    double f = rev - floor(rev);
    sincospi(2.0 * f, &s, &c);
}
// sin^2(pi rev) (for the cancellation-free exp(-j x) - 1)
__device__ __forceinline__ float half_sin(float rev) { return __builtin_amdgcn_sinf(__builtin_amdgcn_fractf(0.5f * rev)); }
__device__ __forceinline__ double half_sin(double rev) { return sinpi(rev); }

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq(double x) { return rsqrt(x); }

// ------------------------------------------------------------------ static self integrals (FP64)
// F(v) = (v^2 + b^2)^(-1/2) and its iterated antiderivatives F1..F4.
struct Anti {
    double f1, f2, f3, f4;
};
__device__ __forceinline__ Anti anti(double v, double b) {
    double s = sqrt(v * v + b * b);
    double ash = asinh(v / b);
    Anti a;
    a.f1 = ash;
    a.f2 = v * ash - s;
    a.f3 = (0.5 * v * v - 0.25 * b * b) * ash - 0.75 * v * s;
    a.f4 = (v * v * v / 6.0 - 0.25 * b * b * v) * ash - (11.0 / 36.0) * s * s * s + (5.0 / 12.0) * b * b * s;
    return a;
}
// K_mn(d) = int_0^1 int_0^1 xi^m xi'^n F(d + xi - xi') dxi' dxi by repeated
// integration by parts (xi: test segment, xi': source segment).  Returns the
// rooftop-half combinations K[a][b] with phi_+ = xi, phi_- = 1 - xi.
__device__ void static_self(const Anti& p1, const Anti& p0, const Anti& m1, double K[2][2]) {
    double k00 = (p1.f2 - p0.f2) - (p0.f2 - m1.f2);
    double k01 = -(p0.f2 - m1.f2) + (p1.f3 - p0.f3) - (p0.f3 - m1.f3);
    double k10 = (p1.f2 - p0.f2) - (p1.f3 - 2.0 * p0.f3 + m1.f3);
    double k11 = (-p0.f2 + p1.f3 - p0.f3) - (-p0.f3 + p1.f4 - p0.f4) + (-m1.f3 + p0.f4 - m1.f4);
    K[0][0] = k11;
    K[0][1] = k10 - k11;
    K[1][0] = k01 - k11;
    K[1][1] = k00 - k10 - k01 + k11;
}

// ------------------------------------------------------------------ self blocks (8 segments)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Self blocks, sampling and assembly.  A wave takes 8 wires; lane (g, d) =
// (lane / 8, lane % 8) runs the Q x Q samples of segment offset d of wire g
// (the block is Toeplitz in d = alpha - beta) and, for d <= 1, adds the
// closed-form static part from its own three FP64 antiderivative values.
// The four rooftop-half terms T_ab(d) of the 8 offsets meet in LDS, and the 8
// lanes of a wire assemble its 49 entries (upper triangle evaluated for both
// (q, q') and (q', q): exactly symmetric), written in place of the diagonal
// block.  No lane idles through a serial step.
constexpr int SELF_WAVES = 4;
template <typename R>
__global__ __launch_bounds__(64 * SELF_WAVES) void k_self(const Wire* __restrict__ wires, int64_t n,
                                                          const int64_t* __restrict__ diag_pos,
                                                          cplx<R>* __restrict__ Z, FillParams prm) {
    using C = cplx<R>;
    __shared__ C Ts[SELF_WAVES][8][NSEG][2][2];   // T_ab(d) of the wave's 8 wires
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int g = lane >> 3, d = lane & 7;
    const int64_t w = ((int64_t)blockIdx.x * SELF_WAVES + wv) * 8 + g;
    const bool live = w < n;
    const Wire wr = wires[live ? w : n - 1];
    const double Dd = wr.len / NSEG;
    const R D = (R)Dd;
    const R a2 = (R)(wr.rad * wr.rad);
    const R inv_lam = (R)prm.inv_lambda;
    const int q = prm.q;
    C m00 = {0, 0}, m01 = {0, 0}, m10 = {0, 0}, m11 = {0, 0};
    for (int kk = 0; kk < q; ++kk) {
        const R xk = (R)prm.xq[kk];
        C s0 = {0, 0}, s1 = {0, 0};
        for (int l = 0; l < q; ++l) {
            const R xl = (R)prm.xq[l];
            const R gl = (R)prm.wq[l];
            R u = D * ((R)d + (xk - xl));
            R r2 = u * u + a2;
            R ir = rsq(r2);
            R rev = r2 * ir * inv_lam;
            R c, sn, gre;
            phase_cs(rev, c, sn);
            if (d <= 1) {   // (exp(-jkR) - 1)/R = (-2 sin^2(kR/2) - j sin kR)/R
                const R hs = half_sin(rev);
                gre = (R)-2 * hs * hs * ir;
            } else {
                gre = c * ir;
            }
            const R gim = -sn * ir;
            s0.re += gl * gre; s0.im += gl * gim;
            s1.re += gl * xl * gre; s1.im += gl * xl * gim;
        }
        const R gk = (R)prm.wq[kk];
        m00 = cadd(m00, cscale(s0, gk));
        m01 = cadd(m01, cscale(s1, gk));
        m10 = cadd(m10, cscale(s0, gk * xk));
        m11 = cadd(m11, cscale(s1, gk * xk));
    }
    const R sc = (R)(Dd * Dd / (4.0 * PI));
    C A[2][2];
    A[0][0] = cscale(m11, sc);
    A[0][1] = cscale(csub(m10, m11), sc);
    A[1][0] = cscale(csub(m01, m11), sc);
    A[1][1] = cscale(cadd(csub(csub(m00, m10), m01), m11), sc);
    if (d <= 1) {   // closed-form static part, antiderivatives at v = d + 1, d, d - 1
        const double b = wr.rad / Dd;
        double K[2][2];
        static_self(anti((double)(d + 1), b), anti((double)d, b), anti((double)(d - 1), b), K);
        for (int a = 0; a < 2; ++a)
            for (int bb = 0; bb < 2; ++bb) A[a][bb].re += (R)(Dd / (4.0 * PI) * K[a][bb]);
    }
    const C B = cadd(cadd(A[0][0], A[0][1]), cadd(A[1][0], A[1][1]));
    const R sz = (R)(1.0 / (prm.k * prm.k * Dd * Dd));
    auto& T = Ts[wv][g];
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb) T[d][a][bb] = csub(A[a][bb], cscale(B, (a == bb ? (R)1 : (R)-1) * sz));
    wave_sync();
    if (!live) return;
    C* Zb = Z + diag_pos[w] * NB2;
    for (int e = d; e < NB2; e += 8) {
        const int qi = e / NB, qj = e % NB;
        const int qa = qi < qj ? qi : qj, qb = qi < qj ? qj : qi;
        C acc = {0, 0};
        for (int da = 0; da < 2; ++da)
            for (int db = 0; db < 2; ++db) {
                const int dd = (qa + da) - (qb + db);
                acc = cadd(acc, dd >= 0 ? T[dd][da][db] : T[-dd][db][da]);
            }
        Zb[e] = acc;
    }
}

// In-place Gauss-Jordan inverse with partial pivoting of one 7 x 7 block held
// in registers (a[i][j]), every index static: the pivot row is found with
// compares and moved with selects, and the column swaps of the pivoting are
// undone the same way at the end.  Returns false for a zero pivot.
template <typename R>
__device__ __forceinline__ bool inverse7_regs(cplx<R> (&a)[NB][NB]) {
    using C = cplx<R>;
    int piv[NB];
#pragma unroll
    for (int p = 0; p < NB; ++p) {
        int b = p;
        R bm = a[p][p].re * a[p][p].re + a[p][p].im * a[p][p].im;
#pragma unroll
        for (int i = p + 1; i < NB; ++i) {
            const R m = a[i][p].re * a[i][p].re + a[i][p].im * a[i][p].im;
            if (m > bm) { bm = m; b = i; }
        }
        piv[p] = b;
        if (!(bm > (R)0)) return false;
#pragma unroll
        for (int i = p + 1; i < NB; ++i) {
            const bool sw = i == b;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const C t = a[p][j];
                a[p][j] = sw ? a[i][j] : t;
                a[i][j] = sw ? t : a[i][j];
            }
        }
        const R inv_m = (R)1 / bm;
        const C ip = {a[p][p].re * inv_m, -a[p][p].im * inv_m};
        a[p][p] = C{1, 0};
#pragma unroll
        for (int j = 0; j < NB; ++j) a[p][j] = cmul(a[p][j], ip);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            if (i == p) continue;
            const C f = a[i][p];
            a[i][p] = C{0, 0};
#pragma unroll
            for (int j = 0; j < NB; ++j) a[i][j] = csub(a[i][j], cmul(f, a[p][j]));
        }
    }
#pragma unroll
    for (int p = NB - 1; p >= 0; --p) {
#pragma unroll
        for (int c = p + 1; c < NB; ++c) {
            const bool sw = c == piv[p];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const C t = a[i][p];
                a[i][p] = sw ? a[i][c] : t;
                a[i][c] = sw ? t : a[i][c];
            }
        }
    }
    return true;
}

// Inverse self blocks (block-diagonal preconditioner of Sec. II-B): one lane
// per wire, WPW wires per wave.  The wave stages its wires' diagonal blocks
// in LDS as A[entry][lane] (consecutive lanes, consecutive words) with
// coalesced loads; each lane inverts its own block by
// Gauss-Jordan with partial pivoting -- in registers for complex64, in place
// in LDS for complex128 (rows swapped in LDS, the column swaps undone at the
// end) -- and the inverses are stored with coalesced writes.
template <typename R, int WPW>
__global__ __launch_bounds__(64) void k_self_inverse(int64_t n, const int64_t* __restrict__ diag_pos,
                                                     const cplx<R>* __restrict__ Z, cplx<R>* __restrict__ Pinv,
                                                     int32_t* __restrict__ status) {
    using C = cplx<R>;
    // one spare column: the staging loops (lanes along the entries of a block)
    // then step 65 words per lane instead of 64, so they do not all hit one bank
    __shared__ C A[NB2][WPW + 1];
    __shared__ int64_t dpos[WPW];
    const int lane = threadIdx.x;
    const int64_t w0 = (int64_t)blockIdx.x * WPW;
    const int nw = (int)(n - w0 < WPW ? n - w0 : WPW);
    if (lane < nw) dpos[lane] = diag_pos[w0 + lane];
    __syncthreads();
    // a fixed trip count unrolled by 8: eight loads of the staging pass in flight per lane
    constexpr int PASSES = (NB2 * WPW + 63) / 64;
#pragma unroll 8
    for (int j = 0; j < PASSES; ++j) {
        const int it = lane + 64 * j;
        const int wl = it / NB2, e = it - wl * NB2;
        if (wl < nw) A[e][wl] = Z[dpos[wl] * NB2 + e];
    }
    __syncthreads();
    if (lane < nw) {
        bool ok = true;
        if constexpr (sizeof(R) == sizeof(float)) {
            C a[NB][NB];
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) a[i][j] = A[i * NB + j][lane];
            ok = inverse7_regs<R>(a);
#pragma unroll
            for (int i = 0; i < NB; ++i)
#pragma unroll
                for (int j = 0; j < NB; ++j) A[i * NB + j][lane] = a[i][j];
        } else {
            int piv[NB];
#pragma unroll
            for (int p = 0; p < NB; ++p) {
                int b = p;
                R bm = A[p * NB + p][lane].re * A[p * NB + p][lane].re +
                       A[p * NB + p][lane].im * A[p * NB + p][lane].im;
#pragma unroll
                for (int i = p + 1; i < NB; ++i) {
                    const C v = A[i * NB + p][lane];
                    const R m = v.re * v.re + v.im * v.im;
                    if (m > bm) { bm = m; b = i; }
                }
                piv[p] = b;
                if (!(bm > (R)0)) { ok = false; break; }
                C rowp[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    rowp[j] = A[b * NB + j][lane];
                    if (b != p) A[b * NB + j][lane] = A[p * NB + j][lane];
                }
                const R inv_m = (R)1 / bm;
                const C ip = {rowp[p].re * inv_m, -rowp[p].im * inv_m};
                rowp[p] = C{1, 0};
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    rowp[j] = cmul(rowp[j], ip);
                    A[p * NB + j][lane] = rowp[j];
                }
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    if (i == p) continue;
                    const C f = A[i * NB + p][lane];
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        const C cur = (j == p) ? C{0, 0} : A[i * NB + j][lane];
                        A[i * NB + j][lane] = csub(cur, cmul(f, rowp[j]));
                    }
                }
            }
            if (ok) {
#pragma unroll
                for (int p = NB - 1; p >= 0; --p) {
                    const int b = piv[p];
                    if (b != p) {
#pragma unroll
                        for (int i = 0; i < NB; ++i) {
                            const C t = A[i * NB + p][lane];
                            A[i * NB + p][lane] = A[i * NB + b][lane];
                            A[i * NB + b][lane] = t;
                        }
                    }
                }
            }
        }
        if (!ok) atomicOr(status, 1);
    }
    __syncthreads();
#pragma unroll 8
    for (int j = 0; j < PASSES; ++j) {
        const int it = lane + 64 * j;
        const int wl = it / NB2, e = it - wl * NB2;
        if (wl < nw) Pinv[(w0 + wl) * NB2 + e] = A[e][wl];
    }
}

// ------------------------------------------------------------------ mutual blocks

template <typename R, int Q>
__global__ __launch_bounds__(256) void k_mutual(const Wire* __restrict__ wires,
                                                const Pair* __restrict__ pairs, int64_t n_pairs,
                                                cplx<R>* __restrict__ Z, FillParams prm) {
    using C = cplx<R>;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform
    const int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    if (e >= n_pairs) return;
    const Pair pr = pairs[e];
    const Wire wi = wires[pr.i];
    const Wire wj = wires[pr.j];
    const int al = lane >> 3, be = lane & 7;

    // FP64 geometry of this segment pair, rounded once to R
    const double Di = wi.len / NSEG, Dj = wj.len / NSEG;
    const double sep[3] = {wj.cx - wi.cx, wj.cy - wi.cy, wj.cz - wi.cz};
    const double s0i = -0.5 * wi.len + al * Di;   // start of segment alpha on wire i
    const double s0j = -0.5 * wj.len + be * Dj;   // start of segment beta on wire j
    // r_i(xi) - r_j(xi') = (s0i t_i - sep - s0j t_j) + xi Di t_i - xi' Dj t_j
    const R bx = (R)(s0i * wi.tx - sep[0] - s0j * wj.tx);
    const R by = (R)(s0i * wi.ty - sep[1] - s0j * wj.ty);
    const R bz = (R)(s0i * wi.tz - sep[2] - s0j * wj.tz);
    const R uix = (R)(Di * wi.tx), uiy = (R)(Di * wi.ty), uiz = (R)(Di * wi.tz);
    const R ujx = (R)(Dj * wj.tx), ujy = (R)(Dj * wj.ty), ujz = (R)(Dj * wj.tz);
    const R a2 = (R)(0.5 * (wi.rad * wi.rad + wj.rad * wj.rad));
    const R inv_lam = (R)prm.inv_lambda;

    R xq[Q], wq[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        xq[k] = (R)prm.xq[k];
        wq[k] = (R)prm.wq[k];
    }
    // source node offsets (relative): -xi'_l Dj t_j
    R px[Q], py[Q], pz[Q];
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        px[l] = bx - xq[l] * ujx;
        py[l] = by - xq[l] * ujy;
        pz[l] = bz - xq[l] * ujz;
    }
    C m00 = {0, 0}, m01 = {0, 0}, m10 = {0, 0}, m11 = {0, 0};
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const R ox = xq[k] * uix, oy = xq[k] * uiy, oz = xq[k] * uiz;
        C s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
        for (int l = 0; l < Q; ++l) {
            R dx = px[l] + ox, dy = py[l] + oy, dz = pz[l] + oz;
            R r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, a2)));
            R ir = rsq(r2);
            R rev = r2 * ir * inv_lam;
            R c, s;
            phase_cs(rev, c, s);
            R gre = c * ir, gim = -s * ir;
            s0.re = fma(wq[l], gre, s0.re);
            s0.im = fma(wq[l], gim, s0.im);
            R wl = wq[l] * xq[l];
            s1.re = fma(wl, gre, s1.re);
            s1.im = fma(wl, gim, s1.im);
        }
        const R wk = wq[k], wkx = wq[k] * xq[k];
        m00.re = fma(wk, s0.re, m00.re); m00.im = fma(wk, s0.im, m00.im);
        m01.re = fma(wk, s1.re, m01.re); m01.im = fma(wk, s1.im, m01.im);
        m10.re = fma(wkx, s0.re, m10.re); m10.im = fma(wkx, s0.im, m10.im);
        m11.re = fma(wkx, s1.re, m11.re); m11.im = fma(wkx, s1.im, m11.im);
    }
    // rooftop halves: A_ab = Di Dj/(4 pi) * moment combination; T_ab = tt A_ab - s_a s_b B/(k^2 Di Dj)
    const R sc = (R)(Di * Dj / (4.0 * PI));
    const R tt = (R)(wi.tx * wj.tx + wi.ty * wj.ty + wi.tz * wj.tz);
    const R sz = (R)(1.0 / (prm.k * prm.k * Di * Dj));
    C App = cscale(m11, sc);
    C Apm = cscale(csub(m10, m11), sc);
    C Amp = cscale(csub(m01, m11), sc);
    C Amm = cscale(cadd(csub(csub(m00, m10), m01), m11), sc);
    C B = cadd(cadd(App, Apm), cadd(Amp, Amm));
    C Bs = cscale(B, sz);
    C Tpp = csub(cscale(App, tt), Bs);
    C Tpm = cadd(cscale(Apm, tt), Bs);
    C Tmp = cadd(cscale(Amp, tt), Bs);
    C Tmm = csub(cscale(Amm, tt), Bs);

    // output lane o < 49 -> (q, q'): needs lanes (q,q') (q,q'+1) (q+1,q') (q+1,q'+1)
    const int o = lane < NB2 ? lane : 0;
    const int qi = o / NB, qj = o % NB;
    const int l00 = qi * 8 + qj;
    C z;
    z.re = __shfl(Tpp.re, l00);
    z.im = __shfl(Tpp.im, l00);
    z.re += __shfl(Tpm.re, l00 + 1);
    z.im += __shfl(Tpm.im, l00 + 1);
    z.re += __shfl(Tmp.re, l00 + 8);
    z.im += __shfl(Tmp.im, l00 + 8);
    z.re += __shfl(Tmm.re, l00 + 9);
    z.im += __shfl(Tmm.im, l00 + 9);
    if (lane < NB2) {
        Z[pr.pos_ij * NB2 + qi * NB + qj] = z;
        Z[pr.pos_ji * NB2 + qj * NB + qi] = z;
    }
}

// ------------------------------------------------------------------ any segment count (20: the paper's own runs)
// The same quadrature and assembly for NS segments (NS - 1 rooftops) where a
// block no longer fits one lane per entry or per segment pair: lanes loop over
// the work items, and the per-item results meet in LDS.

// Self blocks: one wave per wire.  Items (d, k) = (segment offset, test node)
// run in passes of 64 with k fastest, so each pass reduces over the test nodes
// with xor shuffles inside groups of 8 lanes; T_ab(d) goes to LDS, the block
// is assembled from it (Toeplitz, exactly symmetric) and inverted by
// Gauss-Jordan with partial pivoting, lane c < 2 (NS - 1) owning column c of
// the augmented [Z | I].
constexpr int SELFW_WAVES = 2;
template <typename R, int NS>
__global__ __launch_bounds__(64 * SELFW_WAVES) void k_self_w(const Wire* __restrict__ wires, int64_t n,
                                                             const int64_t* __restrict__ diag_pos,
                                                             cplx<R>* __restrict__ Z, cplx<R>* __restrict__ Pinv,
                                                             FillParams prm, int32_t* __restrict__ status) {
    using C = cplx<R>;
    constexpr int NBW = NS - 1, NBW2 = NBW * NBW;
    static_assert(2 * NBW <= 64, "one lane per column of the augmented matrix");
    __shared__ C Ts[SELFW_WAVES][NS][2][2];        // T_ab(d), d = 0..NS-1
    __shared__ C Abs[SELFW_WAVES][NBW][2 * NBW];   // augmented [Z | I]
    __shared__ Anti As[SELFW_WAVES][4];            // static antiderivatives at v = -1, 0, 1, 2
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * SELFW_WAVES + wv;
    if (w >= n) return;   // uniform over the wave
    auto& T = Ts[wv];
    auto& Ab = Abs[wv];
    const Wire wr = wires[w];
    const double Dd = wr.len / NS;
    const R D = (R)Dd;
    const R a2 = (R)(wr.rad * wr.rad);
    const R inv_lam = (R)prm.inv_lambda;
    const int q = prm.q;
    if (lane < 4) As[wv][lane] = anti((double)(lane - 1), wr.rad / Dd);
    wave_sync();
    const int kk = lane & 7;
    for (int d0 = 0; d0 < NS; d0 += 8) {   // wave-uniform passes over 8 offsets
        const int d = d0 + (lane >> 3);
        C m00 = {0, 0}, m01 = {0, 0}, m10 = {0, 0}, m11 = {0, 0};
        if (d < NS && kk < q) {
            const R xk = (R)prm.xq[kk];
            C s0 = {0, 0}, s1 = {0, 0};
            for (int l = 0; l < q; ++l) {
                const R xl = (R)prm.xq[l];
                const R gl = (R)prm.wq[l];
                R u = D * ((R)d + (xk - xl));
                R r2 = u * u + a2;
                R ir = rsq(r2);
                R rev = r2 * ir * inv_lam;
                R gre, gim, c, sn;
                phase_cs(rev, c, sn);
                if (d <= 1) {   // (exp(-jkR) - 1)/R = (-2 sin^2(kR/2) - j sin kR)/R
                    R hs = half_sin(rev);
                    gre = (R)-2 * hs * hs * ir;
                } else {
                    gre = c * ir;
                }
                gim = -sn * ir;
                s0.re += gl * gre; s0.im += gl * gim;
                s1.re += gl * xl * gre; s1.im += gl * xl * gim;
            }
            const R gk = (R)prm.wq[kk];
            m00 = cscale(s0, gk);
            m01 = cscale(s1, gk);
            m10 = cscale(s0, gk * xk);
            m11 = cscale(s1, gk * xk);
        }
        for (int o = 1; o < 8; o <<= 1) {
            m00.re += __shfl_xor(m00.re, o); m00.im += __shfl_xor(m00.im, o);
            m01.re += __shfl_xor(m01.re, o); m01.im += __shfl_xor(m01.im, o);
            m10.re += __shfl_xor(m10.re, o); m10.im += __shfl_xor(m10.im, o);
            m11.re += __shfl_xor(m11.re, o); m11.im += __shfl_xor(m11.im, o);
        }
        if (kk == 0 && d < NS) {
            const R sc = (R)(Dd * Dd / (4.0 * PI));
            C A[2][2];
            A[0][0] = cscale(m11, sc);
            A[0][1] = cscale(csub(m10, m11), sc);
            A[1][0] = cscale(csub(m01, m11), sc);
            A[1][1] = cscale(cadd(csub(csub(m00, m10), m01), m11), sc);
            if (d <= 1) {   // v = d + 1, d, d - 1 sit at As[d + 2], As[d + 1], As[d]
                double K[2][2];
                static_self(As[wv][d + 2], As[wv][d + 1], As[wv][d], K);
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) A[a][b].re += (R)(Dd / (4.0 * PI) * K[a][b]);
            }
            C B = cadd(cadd(A[0][0], A[0][1]), cadd(A[1][0], A[1][1]));
            const R sz = (R)(1.0 / (prm.k * prm.k * Dd * Dd));
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    R sg = (a == b) ? (R)1 : (R)-1;
                    T[d][a][b] = csub(A[a][b], cscale(B, sg * sz));
                }
        }
    }
    wave_sync();
    C* Zb = Z + diag_pos[w] * NBW2;
    for (int e = lane; e < NBW2; e += 64) {
        const int qi = e / NBW, qj = e % NBW;
        const int qa = qi < qj ? qi : qj, qb = qi < qj ? qj : qi;   // upper triangle: exact symmetry
        C acc = {0, 0};
        for (int da = 0; da < 2; ++da)
            for (int db = 0; db < 2; ++db) {
                const int dd = (qa + da) - (qb + db);
                acc = cadd(acc, dd >= 0 ? T[dd][da][db] : T[-dd][db][da]);
            }
        Zb[e] = acc;
        Ab[qi][qj] = acc;
        Ab[qi][NBW + qj] = (qi == qj) ? C{1, 0} : C{0, 0};
    }
    wave_sync();
    if (Pinv == nullptr) return;
    bool singular = false;
    for (int piv = 0; piv < NBW; ++piv) {
        int best = piv;
        R bm = Ab[piv][piv].re * Ab[piv][piv].re + Ab[piv][piv].im * Ab[piv][piv].im;
        for (int r = piv + 1; r < NBW; ++r) {
            R m = Ab[r][piv].re * Ab[r][piv].re + Ab[r][piv].im * Ab[r][piv].im;
            if (m > bm) { bm = m; best = r; }
        }
        if (!(bm > (R)0)) { singular = true; break; }
        const C pv = Ab[best][piv];
        wave_sync();
        if (lane < 2 * NBW) {
            C tmp = Ab[piv][lane];
            Ab[piv][lane] = Ab[best][lane];
            Ab[best][lane] = tmp;
        }
        wave_sync();
        const R inv_m = (R)1 / bm;
        const C ip = {pv.re * inv_m, -pv.im * inv_m};
        C rowp = {0, 0};
        if (lane < 2 * NBW) rowp = cmul(Ab[piv][lane], ip);
        // every lane reads column piv of the rows (after the swap) before any lane overwrites it
        for (int r = 0; r < NBW; ++r) {
            const C f = Ab[r][piv];
            wave_sync();
            if (lane < 2 * NBW) Ab[r][lane] = (r == piv) ? rowp : csub(Ab[r][lane], cmul(f, rowp));
            wave_sync();
        }
    }
    if (singular) {
        if (lane == 0) atomicOr(status, 1);
        return;
    }
    for (int e = lane; e < NBW2; e += 64) Pinv[w * NBW2 + e] = Ab[e / NBW][NBW + e % NBW];
}

// Mutual blocks: one wave per unique pair.  Items = the NS x NS segment pairs
// (alpha, beta), lane l taking items l, l + 64, ...; each runs the Q x Q
// samples and leaves its four rooftop-half terms T_ab in LDS, from which the
// lanes assemble the (NS - 1)^2 block entries (each needs the four segment
// pairs its two rooftops overlap), stored as Z_ij and Z_ji = Z_ij^T.
constexpr int MUTW_WAVES = 2;
template <typename R, int Q, int NS>
__global__ __launch_bounds__(64 * MUTW_WAVES) void k_mutual_w(const Wire* __restrict__ wires,
                                                              const Pair* __restrict__ pairs, int64_t n_pairs,
                                                              cplx<R>* __restrict__ Z, FillParams prm) {
    using C = cplx<R>;
    constexpr int NBW = NS - 1, NBW2 = NBW * NBW;
    __shared__ C Tsh[MUTW_WAVES][NS * NS][4];   // T_pp, T_pm, T_mp, T_mm of segment pair (alpha, beta)
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t e = (int64_t)blockIdx.x * MUTW_WAVES + wv;
    if (e >= n_pairs) return;
    auto& T = Tsh[wv];
    const Pair pr = pairs[e];
    const Wire wi = wires[pr.i];
    const Wire wj = wires[pr.j];
    const double Di = wi.len / NS, Dj = wj.len / NS;
    const double sep[3] = {wj.cx - wi.cx, wj.cy - wi.cy, wj.cz - wi.cz};
    const R uix = (R)(Di * wi.tx), uiy = (R)(Di * wi.ty), uiz = (R)(Di * wi.tz);
    const R ujx = (R)(Dj * wj.tx), ujy = (R)(Dj * wj.ty), ujz = (R)(Dj * wj.tz);
    const R a2 = (R)(0.5 * (wi.rad * wi.rad + wj.rad * wj.rad));
    const R inv_lam = (R)prm.inv_lambda;
    const R sc = (R)(Di * Dj / (4.0 * PI));
    const R tt = (R)(wi.tx * wj.tx + wi.ty * wj.ty + wi.tz * wj.tz);
    const R sz = (R)(1.0 / (prm.k * prm.k * Di * Dj));
    R xq[Q], wq[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        xq[k] = (R)prm.xq[k];
        wq[k] = (R)prm.wq[k];
    }
    for (int it = lane; it < NS * NS; it += 64) {
        const int al = it / NS, be = it % NS;
        const double s0i = -0.5 * wi.len + al * Di;
        const double s0j = -0.5 * wj.len + be * Dj;
        const R bx = (R)(s0i * wi.tx - sep[0] - s0j * wj.tx);
        const R by = (R)(s0i * wi.ty - sep[1] - s0j * wj.ty);
        const R bz = (R)(s0i * wi.tz - sep[2] - s0j * wj.tz);
        C m00 = {0, 0}, m01 = {0, 0}, m10 = {0, 0}, m11 = {0, 0};
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const R ox = xq[k] * uix, oy = xq[k] * uiy, oz = xq[k] * uiz;
            C s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
            for (int l = 0; l < Q; ++l) {
                R dx = (bx - xq[l] * ujx) + ox, dy = (by - xq[l] * ujy) + oy, dz = (bz - xq[l] * ujz) + oz;
                R r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, a2)));
                R ir = rsq(r2);
                R rev = r2 * ir * inv_lam;
                R c, s;
                phase_cs(rev, c, s);
                R gre = c * ir, gim = -s * ir;
                s0.re = fma(wq[l], gre, s0.re);
                s0.im = fma(wq[l], gim, s0.im);
                R wl = wq[l] * xq[l];
                s1.re = fma(wl, gre, s1.re);
                s1.im = fma(wl, gim, s1.im);
            }
            const R wk = wq[k], wkx = wq[k] * xq[k];
            m00.re = fma(wk, s0.re, m00.re); m00.im = fma(wk, s0.im, m00.im);
            m01.re = fma(wk, s1.re, m01.re); m01.im = fma(wk, s1.im, m01.im);
            m10.re = fma(wkx, s0.re, m10.re); m10.im = fma(wkx, s0.im, m10.im);
            m11.re = fma(wkx, s1.re, m11.re); m11.im = fma(wkx, s1.im, m11.im);
        }
        C App = cscale(m11, sc);
        C Apm = cscale(csub(m10, m11), sc);
        C Amp = cscale(csub(m01, m11), sc);
        C Amm = cscale(cadd(csub(csub(m00, m10), m01), m11), sc);
        C Bs = cscale(cadd(cadd(App, Apm), cadd(Amp, Amm)), sz);
        T[it][0] = csub(cscale(App, tt), Bs);
        T[it][1] = cadd(cscale(Apm, tt), Bs);
        T[it][2] = cadd(cscale(Amp, tt), Bs);
        T[it][3] = csub(cscale(Amm, tt), Bs);
    }
    wave_sync();
    for (int o = lane; o < NBW2; o += 64) {
        const int qi = o / NBW, qj = o % NBW;
        const int l00 = qi * NS + qj;
        C z = T[l00][0];
        z = cadd(z, T[l00 + 1][1]);
        z = cadd(z, T[l00 + NS][2]);
        z = cadd(z, T[l00 + NS + 1][3]);
        Z[pr.pos_ij * NBW2 + qi * NBW + qj] = z;
        Z[pr.pos_ji * NBW2 + qj * NBW + qi] = z;
    }
}

// ------------------------------------------------------------------ host

__global__ void k_fill_status(int32_t* __restrict__ status) {
    if (threadIdx.x == 0) status[0] = 0;
}

template <typename R>
static chaff_status fill_impl(Cloud* c, void* Zv, void* Pinv, hipStream_t st) {
    using C = cplx<R>;
    C* Z = static_cast<C*>(Zv);
    FillParams ps{};
    ps.k = 2.0 * PI / c->wavelength;
    ps.inv_lambda = 1.0 / c->wavelength;
    ps.q = c->q_self;
    for (int i = 0; i < MAXQ; ++i) { ps.xq[i] = c->xq_s[i]; ps.wq[i] = c->wq_s[i]; }
    FillParams pm = ps;
    pm.q = c->q_mutual;
    for (int i = 0; i < MAXQ; ++i) { pm.xq[i] = c->xq_m[i]; pm.wq[i] = c->wq_m[i]; }

    hipLaunchKernelGGL(k_fill_status, dim3(1), dim3(64), 0, st, c->d_status);
    CHAFF_LAUNCH_CHECK();
    if (c->nseg == NSEG_PAPER) {   // 20 segments, 19 x 19 blocks
        constexpr int NS = NSEG_PAPER;
        if (c->n_pairs > 0) {
            dim3 grid((unsigned)((c->n_pairs + MUTW_WAVES - 1) / MUTW_WAVES));
            ProfScope ps("fill_mutual", st, 24.0 * NS * NS * c->q_mutual * c->q_mutual * (double)c->n_pairs, true);
            switch (c->q_mutual) {
#define CHAFF_QW(QQ)                                                                                          \
    case QQ:                                                                                                  \
        hipLaunchKernelGGL((k_mutual_w<R, QQ, NS>), grid, dim3(64 * MUTW_WAVES), 0, st, (const Wire*)c->wires, \
                           (const Pair*)c->pairs, c->n_pairs, Z, pm);                                         \
        break;
                CHAFF_QW(1) CHAFF_QW(2) CHAFF_QW(3) CHAFF_QW(4) CHAFF_QW(5) CHAFF_QW(6) CHAFF_QW(7) CHAFF_QW(8)
#undef CHAFF_QW
                default:
                    return fail(CHAFF_EINVAL, "quad_mutual out of range");
            }
            CHAFF_LAUNCH_CHECK();
        }
        {
            ProfScope pss("fill_self", st, 24.0 * NS * c->q_self * c->q_self * (double)c->n, true);
            hipLaunchKernelGGL((k_self_w<R, NS>), dim3((unsigned)((c->n + SELFW_WAVES - 1) / SELFW_WAVES)),
                               dim3(64 * SELFW_WAVES), 0, st, (const Wire*)c->wires, c->n,
                               (const int64_t*)c->diag_pos, Z, static_cast<C*>(Pinv), ps, c->d_status);
        }
        CHAFF_LAUNCH_CHECK();
    } else if (c->n_pairs > 0) {
        const int wpb = 4;
        dim3 grid((unsigned)((c->n_pairs + wpb - 1) / wpb));
        // 24 flops per Green sample, (8 Q)^2 samples per pair
        ProfScope ps("fill_mutual", st, 24.0 * 64.0 * c->q_mutual * c->q_mutual * (double)c->n_pairs, true);
        switch (c->q_mutual) {
#define CHAFF_Q(QQ)                                                                               \
    case QQ:                                                                                      \
        hipLaunchKernelGGL((k_mutual<R, QQ>), grid, dim3(64 * wpb), 0, st, (const Wire*)c->wires, \
                           (const Pair*)c->pairs, c->n_pairs, Z, pm);                             \
        break;
            CHAFF_Q(1) CHAFF_Q(2) CHAFF_Q(3) CHAFF_Q(4) CHAFF_Q(5) CHAFF_Q(6) CHAFF_Q(7) CHAFF_Q(8)
#undef CHAFF_Q
            default:
                return fail(CHAFF_EINVAL, "quad_mutual out of range");
        }
        CHAFF_LAUNCH_CHECK();
    }
    if (c->nseg == NSEG) {
        {
            ProfScope pss("fill_self", st, 24.0 * 8.0 * c->q_self * c->q_self * (double)c->n, true);
            const int64_t wpb = 8 * SELF_WAVES;
            hipLaunchKernelGGL((k_self<R>), dim3((unsigned)((c->n + wpb - 1) / wpb)), dim3(64 * SELF_WAVES), 0, st,
                               (const Wire*)c->wires, c->n, (const int64_t*)c->diag_pos, Z, ps);
        }
        CHAFF_LAUNCH_CHECK();
        if (Pinv) {
            // Gauss-Jordan: about 8 NB^3 flops per block
            ProfScope psi("fill_self_inverse", st,
                          ProfWork{2.0 * NB2 * sizeof(C) * (double)c->n, 8.0 * NB * NB2 * (double)c->n});
            constexpr int WPW = sizeof(R) == 4 ? 64 : 32;
            hipLaunchKernelGGL((k_self_inverse<R, WPW>), dim3((unsigned)((c->n + WPW - 1) / WPW)), dim3(64), 0, st,
                               c->n, (const int64_t*)c->diag_pos, (const C*)Z, static_cast<C*>(Pinv), c->d_status);
        }
    }
    CHAFF_LAUNCH_CHECK();
    if (Pinv) {
        int32_t flag = 0;
        CHAFF_HIP(hipMemcpyAsync(&flag, c->d_status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        CHAFF_HIP(hipStreamSynchronize(st));
        if (flag) return fail(CHAFF_ESINGULAR, "a self block has a zero pivot");
    }
    return CHAFF_OK;
}

chaff_status fill_Z(Cloud* c, chaff_prec prec, void* Z, void* Pinv, hipStream_t st) {
    if (prec == CHAFF_C64) return fill_impl<float>(c, Z, Pinv, st);
    return fill_impl<double>(c, Z, Pinv, st);
}

}  // namespace chaff
