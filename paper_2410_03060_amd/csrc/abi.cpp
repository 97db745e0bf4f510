// extern "C" entry points of libchaff: host-side validation, error text,
// and dispatch to the gfx950 kernels.  Validation never touches the HIP
// runtime, so argument errors are reported on machines without a GPU.
#include <cmath>
#include <cstdio>
#include <exception>
#include <new>

#include "common.hpp"
#include "tune.hpp"

#include <fstream>
#include <sstream>

namespace chaff {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
chaff_status fail(chaff_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

// Gauss-Legendre on [0,1]: Newton iteration on P_q from the Chebyshev guesses.
void gauss_legendre01(int q, double* x, double* w) {
    for (int i = 0; i < MAXQ; ++i) x[i] = w[i] = 0.0;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < q; ++i) {
        double z = std::cos(pi * (i + 0.75) / (q + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pq = q == 1 ? z : p1;
            double pqm1 = q == 1 ? 1.0 : p0;
            dp = q * (z * pq - pqm1) / (z * z - 1.0);
            double dz = pq / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= q; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double pq = q == 1 ? z : p1, pqm1 = q == 1 ? 1.0 : p0;
        dp = q * (z * pq - pqm1) / (z * z - 1.0);
        // node on [-1,1] is z (descending); map to [0,1] ascending
        x[i] = 0.5 * (z + 1.0);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2/((1-z^2)P'^2) on [-1,1], halved
    }
    // ascending order
    for (int i = 0; i < q; ++i)
        for (int j = i + 1; j < q; ++j)
            if (x[j] < x[i]) {
                std::swap(x[i], x[j]);
                std::swap(w[i], w[j]);
            }
}

size_t build_workspace_bytes(int64_t n, int32_t n_clouds, int64_t max_nnzb);
chaff_status build_cloud(const chaff_params* p, const int64_t* cloud_off, const double* center,
                         const double* tangent, const double* length, const double* radius, void* ws,
                         size_t ws_bytes, int64_t* nnzb_out, hipStream_t st, Cloud** out);
chaff_status fill_Z(Cloud* c, chaff_prec prec, void* Z, void* Pinv, hipStream_t st);
// Krylov solvers, products and excitation, one instantiation per rooftop count
#define CHAFF_KRYLOV_DECLS                                                                                          \
    size_t solve_workspace_bytes(const Cloud* c, const chaff_solve_opts* o, int64_t s);                             \
    chaff_status solve(Cloud* c, const chaff_solve_opts* o, const void* Z, const void* Pinv, const double* k_hat,   \
                       const double* e_hat, int64_t s, void* X, void* ws, size_t ws_bytes,                          \
                       chaff_solve_stats* st_out, double* rel_res, hipStream_t st);                                 \
    chaff_status excitation(Cloud* c, const double* k_hat, const double* e_hat, int64_t s, void* U, hipStream_t st); \
    chaff_status spmm_public(Cloud* c, chaff_prec prec, const void* Z, const void* X, void* Y, int64_t s,           \
                             int variant, hipStream_t st);                                                          \
    chaff_status autotune(Cloud* c, chaff_prec prec, const void* Z, void* X, void* Y, int64_t s, int32_t* best,     \
                          double* best_ms, hipStream_t st);
namespace kr7 { CHAFF_KRYLOV_DECLS }
namespace kr19 { CHAFF_KRYLOV_DECLS }
#undef CHAFF_KRYLOV_DECLS
size_t rcs_workspace_bytes(const Cloud* c, int64_t R, int64_t M, int32_t mono);
chaff_status rcs(Cloud* c, const void* Xv, int64_t R, const double* dir, const double* pol, int64_t M, int32_t mono,
                 double* sigma, void* ws, size_t ws_bytes, hipStream_t st);
chaff_status rcs_noalloc(Cloud* c, const void* X, int64_t R, const double* dir, const double* pol, int64_t M,
                         int32_t mono, double* sigma, hipStream_t st);
size_t mlp_workspace_bytes(int64_t rows, int32_t train);
chaff_status mlp_forward(const float* theta, const uint16_t* feat, int64_t M, float* Y, void* ws, size_t ws_bytes,
                         hipStream_t st);
chaff_status mlp_grad(const float* theta, const uint16_t* feat, const float* T, const int64_t* idx, int64_t M,
                      float* grad, float* loss, void* ws, size_t ws_bytes, hipStream_t st);
chaff_status mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t t, float lr, float b1, float b2,
                      float eps, hipStream_t st);
chaff_status mlp_train_step(float* theta, float* m, float* v, int32_t t, float lr, float b1, float b2, float eps,
                            const uint16_t* feat, const float* T, const int64_t* idx, int64_t M, float* loss, void* ws,
                            size_t ws_bytes, hipStream_t st);
chaff_status mlp_features(Cloud* c, const double* k_hat, const double* e_hat, int64_t R, int64_t row0, int64_t n_rows,
                          uint16_t* feat, hipStream_t st);
chaff_status mlp_targets(Cloud* c, chaff_prec prec, const void* Pinv, const double* k_hat, const double* e_hat,
                         int64_t R, const void* X, float* Y, hipStream_t st);
size_t mlp_guess_workspace_bytes(const Cloud* c, int64_t R);
chaff_status mlp_guess(Cloud* c, chaff_prec prec, const void* Pinv, const float* theta, const double* k_hat,
                       const double* e_hat, int64_t R, void* X, void* ws, size_t ws_bytes, hipStream_t st);
int64_t cluster_count(const Cloud* c);
size_t cluster_buffer_bytes(const Cloud* c, chaff_prec prec);
chaff_status cluster_precond(Cloud* c, chaff_prec prec, const void* Z, void* M, hipStream_t st);
chaff_status cluster_apply_public(Cloud* c, chaff_prec prec, const void* M, const void* X, void* Y, int64_t s,
                                  hipStream_t st);
constexpr int NBH_MAX = 8;   // wires per neighbourhood at most (CHAFF_NBHD_MAX)
size_t nbhd_buffer_bytes(const Cloud* c, chaff_prec prec, int size);
chaff_status nbhd_precond(Cloud* c, chaff_prec prec, int size, const void* Z, void* M, bool raw, hipStream_t st);
chaff_status nbhd_mlp_features(Cloud* c, const void* M, int64_t row0, int64_t n_rows, uint16_t* feat, hipStream_t st);
chaff_status nbhd_mlp_targets(Cloud* c, chaff_prec prec, const void* M, const void* Pinv, float* Y, hipStream_t st);
size_t nbhd_mlp_workspace_bytes(const Cloud* c, int size);
chaff_status nbhd_mlp_precond(Cloud* c, chaff_prec prec, int size, const float* theta, const void* Pinv, void* M,
                              void* ws, size_t ws_bytes, hipStream_t st);

}  // namespace chaff

using namespace chaff;

struct chaff_cloud_s {
    Cloud c;
};

#define CHAFF_GUARD_BEGIN try {
#define CHAFF_GUARD_END                                                   \
    }                                                                     \
    catch (const std::bad_alloc&) {                                       \
        return fail(CHAFF_EINVAL, "host allocation failed");              \
    }                                                                     \
    catch (const std::exception& ex) {                                    \
        return fail(CHAFF_EINVAL, std::string("internal error: ") + ex.what()); \
    }                                                                     \
    catch (...) {                                                         \
        return fail(CHAFF_EINVAL, "internal error");                      \
    }

static chaff_status check_params(const chaff_params* p, const int64_t* cloud_off) {
    if (!p) return fail(CHAFF_EINVAL, "params is NULL");
    if (p->n_wires < 1 || p->n_wires > (int64_t)INT32_MAX / 8)
        return fail(CHAFF_EINVAL, "n_wires must be in [1, 2^28)");
    if (p->n_clouds < 1 || p->n_clouds > 65535) return fail(CHAFF_EINVAL, "n_clouds must be in [1, 65535]");
    if (p->n_seg != NSEG && p->n_seg != NSEG_PAPER)
        return fail(CHAFF_EINVAL, "n_seg must be 8 (7 unknowns per wire) or 20 (19 unknowns per wire)");
    if (!(p->wavelength > 0) || !std::isfinite(p->wavelength)) return fail(CHAFF_EINVAL, "wavelength must be > 0");
    if (!(p->d_c >= 0)) return fail(CHAFF_EINVAL, "d_c must be >= 0 (INFINITY for the dense matrix)");
    if (p->quad_mutual < 1 || p->quad_mutual > MAXQ) return fail(CHAFF_EINVAL, "quad_mutual must be in [1, 8]");
    if (p->quad_self < 2 || p->quad_self > MAXQ) return fail(CHAFF_EINVAL, "quad_self must be in [2, 8]");
    if (p->max_nnzb < p->n_wires) return fail(CHAFF_EINVAL, "max_nnzb must be >= n_wires (diagonal blocks)");
    if (!cloud_off) return fail(CHAFF_EINVAL, "cloud_off is NULL");
    if (cloud_off[0] != 0) return fail(CHAFF_EINVAL, "cloud_off[0] must be 0");
    for (int c = 0; c < p->n_clouds; ++c)
        if (cloud_off[c + 1] < cloud_off[c]) return fail(CHAFF_EINVAL, "cloud_off must be non-decreasing");
    if (cloud_off[p->n_clouds] != p->n_wires) return fail(CHAFF_EINVAL, "cloud_off[n_clouds] must equal n_wires");
    return CHAFF_OK;
}

extern "C" {


static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

static chaff_status check_mlp_cloud(chaff_cloud h, const double* k_hat, const double* e_hat, int64_t n_rhs) {
    if (!h || !k_hat || !e_hat) return fail(CHAFF_EINVAL, "NULL argument");
    if (n_rhs < 1) return fail(CHAFF_EINVAL, "n_rhs must be >= 1");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the learned guess needs wires of 8 segments");
    if (!(h->c.d_c > 0) || !std::isfinite(h->c.d_c))
        return fail(CHAFF_EINVAL, "the learned guess needs a finite d_c > 0");
    if (h->c.n > INT64_MAX / n_rhs / CHAFF_MLP_NFEAT) return fail(CHAFF_EINVAL, "n_wires * n_rhs too large");
    return CHAFF_OK;
}

chaff_status chaff_mlp_features(chaff_cloud h, const double* k_hat, const double* e_hat, int64_t n_rhs, int64_t row0,
                                int64_t n_rows, uint16_t* feat, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    chaff_status s = check_mlp_cloud(h, k_hat, e_hat, n_rhs);
    if (s != CHAFF_OK) return s;
    if (!feat || !aligned16(feat)) return fail(CHAFF_EINVAL, "feat must be a 16-byte aligned device pointer");
    if (row0 < 0 || n_rows < 0 || row0 + n_rows > h->c.n * n_rhs)
        return fail(CHAFF_EINVAL, "rows out of range [0, n_wires * n_rhs)");
    return mlp_features(&h->c, k_hat, e_hat, n_rhs, row0, n_rows, feat, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_mlp_targets(chaff_cloud h, chaff_prec prec, const void* Pinv, const double* k_hat,
                               const double* e_hat, int64_t n_rhs, const void* X, float* Y, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    chaff_status s = check_mlp_cloud(h, k_hat, e_hat, n_rhs);
    if (s != CHAFF_OK) return s;
    if (!X || !Y || !Pinv) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "bad prec");
    return mlp_targets(&h->c, prec, Pinv, k_hat, e_hat, n_rhs, X, Y, (hipStream_t)stream);
    CHAFF_GUARD_END
}

size_t chaff_mlp_workspace_bytes(int64_t n_rows, int32_t train) {
    if (n_rows < 1 || n_rows > ((int64_t)1 << 40)) return 0;
    return mlp_workspace_bytes(n_rows, train);
}

chaff_status chaff_mlp_forward(const float* theta, const uint16_t* feat, int64_t n_rows, float* Y, void* ws,
                               size_t ws_bytes, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!theta || !feat || !Y || !ws) return fail(CHAFF_EINVAL, "NULL argument");
    if (!aligned16(feat)) return fail(CHAFF_EINVAL, "feat must be 16-byte aligned");
    if (n_rows < 1 || n_rows > ((int64_t)1 << 40)) return fail(CHAFF_EINVAL, "n_rows out of range");
    if (ws_bytes < mlp_workspace_bytes(n_rows, 0)) return fail(CHAFF_EWORKSPACE, "mlp workspace too small");
    return mlp_forward(theta, feat, n_rows, Y, ws, ws_bytes, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_mlp_grad(const float* theta, const uint16_t* feat, const float* T, const int64_t* idx,
                            int64_t n_rows, float* grad, float* loss, void* ws, size_t ws_bytes, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!theta || !feat || !T || !grad || !ws) return fail(CHAFF_EINVAL, "NULL argument");
    if (!aligned16(feat)) return fail(CHAFF_EINVAL, "feat must be 16-byte aligned");
    if (n_rows < 1 || n_rows > ((int64_t)1 << 40)) return fail(CHAFF_EINVAL, "n_rows out of range");
    if (ws_bytes < mlp_workspace_bytes(n_rows, 1)) return fail(CHAFF_EWORKSPACE, "mlp workspace too small");
    return mlp_grad(theta, feat, T, idx, n_rows, grad, loss, ws, ws_bytes, (hipStream_t)stream);
    CHAFF_GUARD_END
}

static chaff_status check_adam(int32_t t, float lr, float b1, float b2, float eps) {
    if (t < 1) return fail(CHAFF_EINVAL, "Adam step t must be >= 1");
    if (!(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
        return fail(CHAFF_EINVAL, "bad Adam hyper-parameters");
    return CHAFF_OK;
}

chaff_status chaff_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t t, float lr, float beta1,
                            float beta2, float eps, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!theta || !m || !v || !grad) return fail(CHAFF_EINVAL, "NULL argument");
    chaff_status s = check_adam(t, lr, beta1, beta2, eps);
    if (s != CHAFF_OK) return s;
    return mlp_adam(theta, m, v, grad, t, lr, beta1, beta2, eps, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_mlp_train_step(float* theta, float* m, float* v, int32_t t, float lr, float beta1, float beta2,
                                  float eps, const uint16_t* feat, const float* T, const int64_t* idx, int64_t n_rows,
                                  float* loss, void* ws, size_t ws_bytes, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!theta || !m || !v || !feat || !T || !ws) return fail(CHAFF_EINVAL, "NULL argument");
    if (!aligned16(feat)) return fail(CHAFF_EINVAL, "feat must be 16-byte aligned");
    if (n_rows < 1 || n_rows > ((int64_t)1 << 40)) return fail(CHAFF_EINVAL, "n_rows out of range");
    chaff_status s = check_adam(t, lr, beta1, beta2, eps);
    if (s != CHAFF_OK) return s;
    if (ws_bytes < mlp_workspace_bytes(n_rows, 1)) return fail(CHAFF_EWORKSPACE, "mlp workspace too small");
    return mlp_train_step(theta, m, v, t, lr, beta1, beta2, eps, feat, T, idx, n_rows, loss, ws, ws_bytes,
                          (hipStream_t)stream);
    CHAFF_GUARD_END
}

size_t chaff_mlp_guess_workspace_bytes(chaff_cloud h, int64_t n_rhs) {
    if (!h || n_rhs < 1) return 0;
    return mlp_guess_workspace_bytes(&h->c, n_rhs);
}

chaff_status chaff_mlp_guess(chaff_cloud h, chaff_prec prec, const void* Pinv, const float* theta,
                             const double* k_hat, const double* e_hat, int64_t n_rhs, void* X, void* ws,
                             size_t ws_bytes, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    chaff_status s = check_mlp_cloud(h, k_hat, e_hat, n_rhs);
    if (s != CHAFF_OK) return s;
    if (!theta || !X || !ws || !Pinv) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "bad prec");
    if (ws_bytes < mlp_guess_workspace_bytes(&h->c, n_rhs))
        return fail(CHAFF_EWORKSPACE, "mlp guess workspace too small");
    return mlp_guess(&h->c, prec, Pinv, theta, k_hat, e_hat, n_rhs, X, ws, ws_bytes, (hipStream_t)stream);
    CHAFF_GUARD_END
}

const char* chaff_last_error(void) { return g_last_error.c_str(); }
const char* chaff_version(void) { return "chaff-gfx950 1.0"; }

size_t chaff_build_workspace_bytes(int64_t n_wires, int32_t n_clouds, int64_t max_nnzb) {
    if (n_wires < 1 || n_clouds < 1 || max_nnzb < n_wires) return 0;
    return build_workspace_bytes(n_wires, n_clouds, max_nnzb);
}

chaff_status chaff_build_cloud(const chaff_params* p, const int64_t* cloud_off, const double* center,
                               const double* tangent, const double* length, const double* radius, void* ws,
                               size_t ws_bytes, int64_t* nnzb, chaff_stream stream, chaff_cloud* out) {
    CHAFF_GUARD_BEGIN
    chaff_status s = check_params(p, cloud_off);
    if (s != CHAFF_OK) return s;
    if (!center || !tangent || !length || !radius) return fail(CHAFF_EINVAL, "geometry pointer is NULL");
    if (!nnzb || !out) return fail(CHAFF_EINVAL, "nnzb/out is NULL");
    if (!ws) return fail(CHAFF_EINVAL, "workspace is NULL");
    *out = nullptr;
    *nnzb = 0;
    size_t need = build_workspace_bytes(p->n_wires, p->n_clouds, p->max_nnzb);
    if (ws_bytes < need)
        return fail(CHAFF_EWORKSPACE, "build workspace too small: need " + std::to_string(need));
    Cloud* c = nullptr;
    s = build_cloud(p, cloud_off, center, tangent, length, radius, ws, ws_bytes, nnzb, (hipStream_t)stream, &c);
    if (s != CHAFF_OK) return s;
    chaff_cloud_s* h = new chaff_cloud_s;
    h->c = *c;
    delete c;
    *out = h;
    return CHAFF_OK;
    CHAFF_GUARD_END
}

chaff_status chaff_get_info(chaff_cloud h, chaff_cloud_info* info) {
    if (!h || !info) return fail(CHAFF_EINVAL, "NULL handle/info");
    const Cloud& c = h->c;
    info->n_wires = c.n;
    info->nnzb = c.nnzb;
    info->n_pairs = c.n_pairs;
    info->n_clouds = c.n_clouds;
    info->n_seg = c.nseg;
    info->wavelength = c.wavelength;
    info->d_c = c.d_c;
    info->row_ptr = c.row_ptr;
    info->col_idx = c.col_idx;
    info->perm = c.perm;
    info->diag_pos = c.diag_pos;
    return CHAFF_OK;
}

chaff_status chaff_fill_Z(chaff_cloud h, chaff_prec prec, void* Z, void* Pinv, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h) return fail(CHAFF_EINVAL, "NULL handle");
    if (!Z) return fail(CHAFF_EINVAL, "Z is NULL");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    return fill_Z(&h->c, prec, Z, Pinv, (hipStream_t)stream);
    CHAFF_GUARD_END
}

static chaff_status check_opts(const chaff_solve_opts* o) {
    if (!o) return fail(CHAFF_EINVAL, "opts is NULL");
    if (!(o->tol > 0) || !(o->tol < 1)) return fail(CHAFF_EINVAL, "tol must be in (0, 1)");
    if (!(o->inner_tol > 0) || !(o->inner_tol < 1)) return fail(CHAFF_EINVAL, "inner_tol must be in (0, 1)");
    const bool restarted = o->method == CHAFF_GMRES || o->method == CHAFF_GCR;
    if (o->restart < 1 || (restarted && o->restart > 200))
        return fail(CHAFF_EINVAL, "restart must be in [1, 200] (GMRES, GCR) or >= 1 (COCG)");
    if (o->max_cycles < 1) return fail(CHAFF_EINVAL, "max_cycles must be >= 1");
    if (o->use_x0 < 0 || o->use_x0 > 2) return fail(CHAFF_EINVAL, "use_x0 must be 0, 1 or 2");
    if (o->prec != CHAFF_C64 && o->prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    if (o->spmm_variant < -1 || o->spmm_variant > 7) return fail(CHAFF_EINVAL, "spmm_variant must be in [-1, 7]");
    if (o->method != CHAFF_GMRES && o->method != CHAFF_COCG && o->method != CHAFF_COCG_RR && o->method != CHAFF_GCR)
        return fail(CHAFF_EINVAL, "method must be CHAFF_GMRES, CHAFF_COCG, CHAFF_COCG_RR or CHAFF_GCR");
    if (!restarted && o->restart > 1000000) return fail(CHAFF_EINVAL, "restart too large");
    if (o->reserved != 0) return fail(CHAFF_EINVAL, "reserved must be 0");
    if (o->precond != CHAFF_PRECOND_BLOCK && o->precond != CHAFF_PRECOND_CLUSTER && o->precond != CHAFF_PRECOND_NBHD)
        return fail(CHAFF_EINVAL, "precond must be CHAFF_PRECOND_BLOCK, CHAFF_PRECOND_CLUSTER or CHAFF_PRECOND_NBHD");
    return CHAFF_OK;
}

size_t chaff_solve_workspace_bytes(chaff_cloud h, const chaff_solve_opts* o, int64_t n_rhs) {
    if (!h || !o || n_rhs < 1 || check_opts(o) != CHAFF_OK) return 0;
    return h->c.nseg == NSEG ? kr7::solve_workspace_bytes(&h->c, o, n_rhs)
                             : kr19::solve_workspace_bytes(&h->c, o, n_rhs);
}

chaff_status chaff_solve(chaff_cloud h, const chaff_solve_opts* o, const void* Z, const void* Pinv,
                         const double* k_hat, const double* e_hat, int64_t n_rhs, void* X, void* ws, size_t ws_bytes,
                         chaff_solve_stats* st, double* rel_res, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h) return fail(CHAFF_EINVAL, "NULL handle");
    chaff_status s = check_opts(o);
    if (s != CHAFF_OK) return s;
    if (!Z || !Pinv) return fail(CHAFF_EINVAL, "Z and Pinv are required");
    if (o->precond == CHAFF_PRECOND_CLUSTER && ((uintptr_t)Pinv % 256) != 0)
        return fail(CHAFF_EINVAL, "the cluster preconditioner buffer must be 256-byte aligned");
    if (o->precond == CHAFF_PRECOND_NBHD && ((uintptr_t)Pinv % 256) != 0)
        return fail(CHAFF_EINVAL, "the neighbourhood-inverse preconditioner buffer must be 256-byte aligned");
    if (!k_hat || !e_hat || !X || !ws) return fail(CHAFF_EINVAL, "NULL k_hat/e_hat/X/ws");
    if (n_rhs < 1 || n_rhs > 65535) return fail(CHAFF_EINVAL, "n_rhs must be in [1, 65535]");
    if (h->c.nseg != NSEG && o->precond == CHAFF_PRECOND_CLUSTER)
        return fail(CHAFF_EINVAL, "the cluster preconditioner needs wires of 8 segments");
    if (h->c.nseg != NSEG && o->precond == CHAFF_PRECOND_NBHD)
        return fail(CHAFF_EINVAL, "the neighbourhood-inverse preconditioner needs wires of 8 segments");
    const bool k7 = h->c.nseg == NSEG;
    size_t need = k7 ? kr7::solve_workspace_bytes(&h->c, o, n_rhs) : kr19::solve_workspace_bytes(&h->c, o, n_rhs);
    if (ws_bytes < need) return fail(CHAFF_EWORKSPACE, "solve workspace too small: need " + std::to_string(need));
    if (k7) return kr7::solve(&h->c, o, Z, Pinv, k_hat, e_hat, n_rhs, X, ws, ws_bytes, st, rel_res, (hipStream_t)stream);
    return kr19::solve(&h->c, o, Z, Pinv, k_hat, e_hat, n_rhs, X, ws, ws_bytes, st, rel_res, (hipStream_t)stream);
    CHAFF_GUARD_END
}

int64_t chaff_cluster_count(chaff_cloud h) { return h && h->c.nseg == NSEG ? cluster_count(&h->c) : -1; }

size_t chaff_cluster_precond_bytes(chaff_cloud h, chaff_prec prec) {
    if (!h || h->c.nseg != NSEG || (prec != CHAFF_C64 && prec != CHAFF_C128)) return 0;
    return cluster_buffer_bytes(&h->c, prec);
}

chaff_status chaff_cluster_precond(chaff_cloud h, chaff_prec prec, const void* Z, void* M, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !Z || !M) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    if (((uintptr_t)M % 256) != 0) return fail(CHAFF_EINVAL, "M must be 256-byte aligned");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the cluster preconditioner needs wires of 8 segments");
    return cluster_precond(&h->c, prec, Z, M, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_cluster_apply(chaff_cloud h, chaff_prec prec, const void* M, const void* X, void* Y, int64_t s,
                                 chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !M || !X || !Y) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    if (s < 1 || s > 65535) return fail(CHAFF_EINVAL, "s must be in [1, 65535]");
    if (((uintptr_t)M % 256) != 0) return fail(CHAFF_EINVAL, "M must be 256-byte aligned");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the cluster preconditioner needs wires of 8 segments");
    return cluster_apply_public(&h->c, prec, M, X, Y, s, (hipStream_t)stream);
    CHAFF_GUARD_END
}

size_t chaff_nbhd_precond_bytes(chaff_cloud h, chaff_prec prec, int32_t size) {
    if (!h || (prec != CHAFF_C64 && prec != CHAFF_C128) || size < 1 || size > NBH_MAX || h->c.nseg != NSEG) return 0;
    return nbhd_buffer_bytes(&h->c, prec, size);
}

chaff_status chaff_nbhd_precond(chaff_cloud h, chaff_prec prec, int32_t size, const void* Z, void* M,
                                chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !Z || !M) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    if (size < 1 || size > NBH_MAX) return fail(CHAFF_EINVAL, "size must be in [1, CHAFF_NBHD_MAX]");
    if (((uintptr_t)M % 256) != 0) return fail(CHAFF_EINVAL, "M must be 256-byte aligned");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the neighbourhood-inverse preconditioner needs wires of 8 segments");
    return nbhd_precond(&h->c, prec, size, Z, M, false, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_nbhd_raw_rows(chaff_cloud h, chaff_prec prec, int32_t size, const void* Z, void* M,
                                 chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !Z || !M) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    if (size < 1 || size > NBH_MAX) return fail(CHAFF_EINVAL, "size must be in [1, CHAFF_NBHD_MAX]");
    if (((uintptr_t)M % 256) != 0) return fail(CHAFF_EINVAL, "M must be 256-byte aligned");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the neighbourhood-inverse preconditioner needs wires of 8 segments");
    return nbhd_precond(&h->c, prec, size, Z, M, true, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_nbhd_mlp_features(chaff_cloud h, const void* M, int64_t row0, int64_t n_rows, uint16_t* feat,
                                     chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !M || (!feat && n_rows > 0)) return fail(CHAFF_EINVAL, "NULL argument");
    if (row0 < 0 || n_rows < 0) return fail(CHAFF_EINVAL, "row0 and n_rows must be >= 0");
    if (((uintptr_t)M % 256) != 0) return fail(CHAFF_EINVAL, "M must be 256-byte aligned");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the learned preconditioner needs wires of 8 segments");
    if (!std::isfinite(h->c.d_c)) return fail(CHAFF_EINVAL, "the learned preconditioner needs a finite d_c");
    return nbhd_mlp_features(&h->c, M, row0, n_rows, feat, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_nbhd_mlp_targets(chaff_cloud h, chaff_prec prec, const void* M, const void* Pinv, float* Y,
                                    chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !M || !Pinv || !Y) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    if (((uintptr_t)M % 256) != 0) return fail(CHAFF_EINVAL, "M must be 256-byte aligned");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the learned preconditioner needs wires of 8 segments");
    return nbhd_mlp_targets(&h->c, prec, M, Pinv, Y, (hipStream_t)stream);
    CHAFF_GUARD_END
}

size_t chaff_nbhd_mlp_workspace_bytes(chaff_cloud h, int32_t size) {
    if (!h || size < 1 || size > NBH_MAX || h->c.nseg != NSEG) return 0;
    return nbhd_mlp_workspace_bytes(&h->c, size);
}

chaff_status chaff_nbhd_mlp_precond(chaff_cloud h, chaff_prec prec, int32_t size, const float* theta,
                                    const void* Pinv, void* M, void* ws, size_t ws_bytes, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !theta || !Pinv || !M || !ws) return fail(CHAFF_EINVAL, "NULL argument");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "prec must be CHAFF_C64 or CHAFF_C128");
    if (size < 1 || size > NBH_MAX) return fail(CHAFF_EINVAL, "size must be in [1, CHAFF_NBHD_MAX]");
    if (((uintptr_t)M % 256) != 0) return fail(CHAFF_EINVAL, "M must be 256-byte aligned");
    if (h->c.nseg != NSEG) return fail(CHAFF_EINVAL, "the learned preconditioner needs wires of 8 segments");
    if (!std::isfinite(h->c.d_c)) return fail(CHAFF_EINVAL, "the learned preconditioner needs a finite d_c");
    const size_t need = nbhd_mlp_workspace_bytes(&h->c, size);
    if (ws_bytes < need) return fail(CHAFF_EWORKSPACE, "learned preconditioner workspace too small: need " +
                                                           std::to_string(need));
    return nbhd_mlp_precond(&h->c, prec, size, theta, Pinv, M, ws, ws_bytes, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_excitation(chaff_cloud h, const double* k_hat, const double* e_hat, int64_t n_rhs, void* U,
                              chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !k_hat || !e_hat || !U) return fail(CHAFF_EINVAL, "NULL argument");
    if (n_rhs < 1) return fail(CHAFF_EINVAL, "n_rhs must be >= 1");
    if (h->c.nseg == NSEG) return kr7::excitation(&h->c, k_hat, e_hat, n_rhs, U, (hipStream_t)stream);
    return kr19::excitation(&h->c, k_hat, e_hat, n_rhs, U, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_spmm(chaff_cloud h, chaff_prec prec, const void* Z, const void* X, void* Y, int64_t s,
                        int32_t variant, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !Z || !X || !Y) return fail(CHAFF_EINVAL, "NULL argument");
    if (s < 1 || s > 65535) return fail(CHAFF_EINVAL, "s must be in [1, 65535]");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "bad prec");
    if (variant < -1 || variant > 7) return fail(CHAFF_EINVAL, "variant must be in [-1, 7]");
    if (h->c.nseg == NSEG) return kr7::spmm_public(&h->c, prec, Z, X, Y, s, variant, (hipStream_t)stream);
    return kr19::spmm_public(&h->c, prec, Z, X, Y, s, variant, (hipStream_t)stream);
    CHAFF_GUARD_END
}

size_t chaff_rcs_workspace_bytes(chaff_cloud h, int64_t n_rhs, int64_t n_dirs, int32_t monostatic) {
    if (!h || n_rhs < 1 || n_dirs < 1) return 0;
    return rcs_workspace_bytes(&h->c, n_rhs, n_dirs, monostatic);
}

chaff_status chaff_rcs(chaff_cloud h, const void* X, int64_t n_rhs, const double* obs_dir, const double* obs_pol,
                       int64_t n_dirs, int32_t monostatic, double* sigma, void* ws, size_t ws_bytes,
                       chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !X || !obs_dir || !obs_pol || !sigma || !ws) return fail(CHAFF_EINVAL, "NULL argument");
    if (n_rhs < 1 || n_dirs < 1) return fail(CHAFF_EINVAL, "n_rhs and n_dirs must be >= 1");
    if (monostatic && n_dirs != n_rhs) return fail(CHAFF_EINVAL, "monostatic needs n_dirs == n_rhs");
    if (!monostatic && n_rhs > 65535) return fail(CHAFF_EINVAL, "bistatic n_rhs must be <= 65535");
    size_t need = rcs_workspace_bytes(&h->c, n_rhs, n_dirs, monostatic);
    if (ws_bytes < need) return fail(CHAFF_EWORKSPACE, "rcs workspace too small: need " + std::to_string(need));
    return rcs(&h->c, X, n_rhs, obs_dir, obs_pol, n_dirs, monostatic, sigma, ws, ws_bytes, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_rcs_noalloc(chaff_cloud h, const void* X, int64_t n_rhs, const double* obs_dir,
                               const double* obs_pol, int64_t n_dirs, int32_t monostatic, double* sigma,
                               chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !X || !obs_dir || !obs_pol || !sigma) return fail(CHAFF_EINVAL, "NULL argument");
    if (n_rhs < 1 || n_dirs < 1) return fail(CHAFF_EINVAL, "n_rhs and n_dirs must be >= 1");
    if (monostatic && n_dirs != n_rhs) return fail(CHAFF_EINVAL, "monostatic needs n_dirs == n_rhs");
    if (!monostatic && n_rhs > 65535) return fail(CHAFF_EINVAL, "bistatic n_rhs must be <= 65535");
    return rcs_noalloc(&h->c, X, n_rhs, obs_dir, obs_pol, n_dirs, monostatic, sigma, (hipStream_t)stream);
    CHAFF_GUARD_END
}

chaff_status chaff_autotune(chaff_cloud h, chaff_prec prec, const void* Z, void* X, void* Y, int64_t s,
                            int32_t* best_variant, double* best_ms, chaff_stream stream) {
    CHAFF_GUARD_BEGIN
    if (!h || !Z || !X || !Y) return fail(CHAFF_EINVAL, "NULL argument");
    if (s < 1 || s > 65535) return fail(CHAFF_EINVAL, "s must be in [1, 65535]");
    if (prec != CHAFF_C64 && prec != CHAFF_C128) return fail(CHAFF_EINVAL, "bad prec");
    if (h->c.nseg == NSEG) return kr7::autotune(&h->c, prec, Z, X, Y, s, best_variant, best_ms, (hipStream_t)stream);
    return kr19::autotune(&h->c, prec, Z, X, Y, s, best_variant, best_ms, (hipStream_t)stream);
    CHAFF_GUARD_END
}

int32_t chaff_tune_report(char* buf, int32_t len) {
    const std::string out = tune_json();
    if (buf && len > 0) {
        std::strncpy(buf, out.c_str(), (size_t)len - 1);
        buf[len - 1] = 0;
    }
    return (int32_t)out.size() + 1;
}

chaff_status chaff_tune_save(const char* path) {
    CHAFF_GUARD_BEGIN
    if (!path) return fail(CHAFF_EINVAL, "path is NULL");
    std::ofstream f(path, std::ios::out | std::ios::trunc);
    if (!f) return fail(CHAFF_EINVAL, std::string("cannot write ") + path);
    f << tune_json() << "\n";
    if (!f) return fail(CHAFF_EINVAL, std::string("write failed: ") + path);
    return CHAFF_OK;
    CHAFF_GUARD_END
}

chaff_status chaff_tune_load(const char* path, int32_t* n_entries) {
    CHAFF_GUARD_BEGIN
    if (!path) return fail(CHAFF_EINVAL, "path is NULL");
    std::ifstream f(path);
    if (!f) return fail(CHAFF_EINVAL, std::string("cannot read ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    const int n = tune_merge_json(ss.str());
    if (n < 0) return fail(CHAFF_EINVAL, std::string("not a tuning table: ") + path);
    if (n_entries) *n_entries = n;
    return CHAFF_OK;
    CHAFF_GUARD_END
}

void chaff_destroy(chaff_cloud h) { delete h; }

}  // extern "C"
