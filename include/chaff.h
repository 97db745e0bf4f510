/*
 * chaff.h -- C ABI of the MI355X (gfx950) hot path of the sparsified thin-wire
 * method of moments for chaff clouds (S-NFC: sparsification via neglecting
 * far-field coupling).
 *
 * Problem statement (Sec. II-A): N thin perfectly conducting straight wires of
 * arbitrary centre, orientation, length and radius are illuminated by plane
 * waves.  Each wire is cut into n_seg equal segments carrying n_seg - 1
 * rooftop unknowns (eq. 2 and its footnote): n_seg = 8 (7 unknowns), or
 * n_seg = 20 (19 unknowns), the discretisation of the paper's own runs.
 * The Galerkin EFIE system Z x = u (eqs. 3-8) is kept only on wire pairs
 * whose centroid distance is <= d_c (eq. 9) and solved iteratively with a
 * block-diagonal preconditioner (Sec. II-B); the far-field functional then
 * gives monostatic and bistatic radar cross sections (Sec. III).
 *
 * Conventions shared by every call
 *  - Time convention exp(+j w t); G(R) = exp(-j k R)/(4 pi R) with the thin-wire
 *    reduced distance R = sqrt(|r - r'|^2 + a^2) between wire axes
 *    (a^2 = (a_p^2 + a_p'^2)/2 between wires of different radius).
 *  - Units are metres; only the wavelength enters (k = 2 pi / wavelength).
 *  - Unknown order is wire-major in the CALLER's wire order:
 *    n = p*NB + q, q = 0..NB-1 counted from the -L/2 end along the tangent,
 *    NB = n_seg - 1 unknowns per wire.  Multi-RHS vectors are row-major
 *    [N*NB][R] (element (n, r) at n*R + r).  Blocks are NB x NB.
 *  - x is the solution of Z x = u with u the tested incident field
 *    u_n = int L_n (t_n . e) exp(-j k k_hat . r) ds (eq. 4 without its
 *    -(j/(w mu0)) factor).  The physical current is -(j/(w mu0)) x, and for a
 *    unit-amplitude wave sigma = |w^T x|^2 / (4 pi), w the far-field weights.
 *  - Complex numbers are interleaved (re, im): CHAFF_C64 = 2 x float,
 *    CHAFF_C128 = 2 x double.
 *  - Pointers are DEVICE pointers unless marked [host].  The library never
 *    allocates device memory: data-dependent scratch is a caller workspace
 *    whose size is queried first.  Every call is asynchronous on `stream`
 *    (a hipStream_t) except where a host read-back is stated.
 *  - Errors: every entry point returns a chaff_status; inputs are validated
 *    on the host before any launch; no C++ exception crosses the ABI; the
 *    text of the last error of the calling thread is chaff_last_error().
 */
#ifndef CHAFF_H
#define CHAFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

struct ihipStream_t;                  /* hipStream_t is struct ihipStream_t* */
typedef struct ihipStream_t* chaff_stream;

typedef enum {
    CHAFF_OK = 0,
    CHAFF_EINVAL = -1,       /* bad argument (null pointer, size, non-unit tangent ...) */
    CHAFF_EWORKSPACE = -2,   /* workspace too small / pattern capacity exceeded */
    CHAFF_EHIP = -3,         /* a HIP runtime call failed */
    CHAFF_ESINGULAR = -4,    /* a self block could not be inverted */
    CHAFF_ENOCONV = -5       /* solver hit its iteration cap, or a recurrence broke down and left a
                                system's solution non-finite (its relative residual reads +inf);
                                X holds the last iterate */
} chaff_status;

typedef enum { CHAFF_C64 = 0, CHAFF_C128 = 1 } chaff_prec;

typedef struct chaff_cloud_s* chaff_cloud;   /* opaque handle, host memory owned by the library */

#define CHAFF_NSEG 8          /* segments per wire of the default discretisation */
#define CHAFF_NB 7            /* its unknowns per wire */
#define CHAFF_NSEG_PAPER 20   /* the paper's own discretisation: 19 unknowns per wire */

typedef struct {
    int64_t n_wires;          /* total wires over all clouds, >= 1 */
    int32_t n_clouds;         /* independent clouds, >= 1 (pairs never cross clouds) */
    int32_t n_seg;            /* CHAFF_NSEG (8) or CHAFF_NSEG_PAPER (20); the cluster
                                 preconditioner and the learned guess need 8 */
    double  wavelength;       /* metres, > 0 */
    double  d_c;              /* coupling threshold (eq. 9), metres, >= 0; INFINITY = dense */
    int32_t quad_mutual;      /* Gauss-Legendre nodes per segment, different wires (1..8; 4) */
    int32_t quad_self;        /* Gauss-Legendre nodes per segment, same wire (2..8; 8) */
    int64_t max_nnzb;         /* capacity of the block pattern held in the build workspace */
} chaff_params;

/* ------------------------------------------------------------------ build
 * Neighbour search (eq. 9): stored blocks are the diagonal plus every ordered
 * pair (p, p') of one cloud with ((dx*dx + dy*dy) + dz*dz) <= d_c*d_c in
 * IEEE double without fused multiply-add (dx = c_p'.x - c_p.x, ...).
 * Wires are reordered internally along a Morton curve of a cell grid
 * (cell side >= d_c); the block pattern (CSR of NB x NB blocks) is stored in that
 * internal order and its permutation is returned by chaff_get_info.
 *
 * chaff_build_workspace_bytes: [host only] bytes the build workspace needs.
 * chaff_build_cloud:
 *   cloud_off  [host] [n_clouds+1] wire offsets of the clouds, cloud_off[0]=0,
 *              non-decreasing, cloud_off[n_clouds] = n_wires.
 *   center [N][3], tangent [N][3] (unit, |t|^2 within 1e-10 of 1),
 *   length [N] (> 0), radius [N] (> 0, < length/8): double, device.
 *   ws / ws_bytes: device workspace of at least chaff_build_workspace_bytes;
 *              it holds the cloud's internal arrays and must stay allocated
 *              and untouched until chaff_destroy.  The geometry arrays may be
 *              freed after the call.
 *   nnzb       [host out] number of stored blocks.  If it exceeds
 *              p->max_nnzb the call returns CHAFF_EWORKSPACE with *nnzb set
 *              and no handle; call again with a larger capacity.
 *   out        [host out] the handle.
 *   Synchronises `stream` twice (grid bounds and block count read-back).
 */
size_t chaff_build_workspace_bytes(int64_t n_wires, int32_t n_clouds, int64_t max_nnzb);
chaff_status chaff_build_cloud(const chaff_params* p, const int64_t* cloud_off,
                               const double* center, const double* tangent,
                               const double* length, const double* radius,
                               void* ws, size_t ws_bytes, int64_t* nnzb,
                               chaff_stream stream, chaff_cloud* out);

typedef struct {
    int64_t n_wires, nnzb, n_pairs;      /* n_pairs = unique off-diagonal pairs (p < p') */
    int32_t n_clouds, n_seg;
    double  wavelength, d_c;
    const int64_t* row_ptr;              /* [N+1] device, internal order */
    const int32_t* col_idx;              /* [nnzb] device, internal wire indices, ascending per row */
    const int32_t* perm;                 /* [N] device: internal wire i is caller wire perm[i] */
    const int64_t* diag_pos;             /* [N] device: block index of (i, i) */
} chaff_cloud_info;
chaff_status chaff_get_info(chaff_cloud c, chaff_cloud_info* info /* [host out] */);

/* ------------------------------------------------------------------ fill
 * Galerkin impedance blocks (eqs. 5-8) on the stored pattern, with the
 * rooftop assembly of Sec. II-A: tensor Gauss-Legendre per segment pair
 * (quad_mutual nodes between wires, quad_self on one wire); on one wire the
 * static part 1/(4 pi R) of touching and identical segments is integrated in
 * closed form ("analytic singularity extraction").  Z = Z^T block-wise: each
 * unique pair is computed once and stored twice.
 *   Z    [nnzb][NB][NB] complex (prec), internal block order, row-major blocks.
 *   Pinv [N][NB][NB] complex (prec) or NULL: inverse of every self block
 *        (block-diagonal preconditioner of Sec. II-B), internal wire order.
 * Returns CHAFF_ESINGULAR (after the stream completes) if a self block has a
 * zero pivot.
 */
chaff_status chaff_fill_Z(chaff_cloud c, chaff_prec prec, void* Z, void* Pinv,
                          chaff_stream stream);

/* ------------------------------------------------------------------ solve
 * Excitation (eq. 4) for R plane waves, then a preconditioned Krylov solve of
 * the S-NFC system, one independent system per (cloud, RHS), all advanced in
 * lockstep so each sparse product serves every right-hand side.  The Krylov
 * method of every cycle is o->method: restarted GMRES(m), COCG (two forms) or
 * GCR(m), the solver of Sec. II-B (see chaff_method).  The preconditioner is
 * o->precond: the inverse self blocks (block-diagonal preconditioner of
 * Sec. II-B) or the cluster inverses of chaff_cluster_precond; GMRES and GCR
 * apply it on the right, COCG as the symmetric M in z = M r.  With prec =
 * CHAFF_C64 the Krylov work is complex FP32 and every cycle is an
 * iterative-refinement sweep against the FP64 true residual u - Z x (Z the
 * stored matrix, FP64 accumulation).  With CHAFF_C128 everything is FP64.
 * Stops when every system has ||u - Z x||_2 <= tol * ||u||_2 over its
 * cloud's rows.
 */
typedef struct {
    double  tol;              /* relative FP64 residual target per system (1e-6) */
    double  inner_tol;        /* relative reduction asked of one FP32 cycle (1e-4) */
    int32_t restart;          /* GMRES(m) / GCR(m) cycle length, 1..200 (30); COCG: step cap per cycle */
    int32_t max_cycles;       /* restart/refinement cycles (50) */
    int32_t use_x0;           /* 0: x0 = 0; 1: X holds an initial guess on entry;
                                 2: preconditioner guess x0 = P u (P the preconditioner
                                    passed as Pinv: block, cluster or neighbourhood) */
    int32_t prec;             /* chaff_prec of Z, Pinv and the Krylov vectors */
    int32_t spmm_variant;     /* -1: tuned (chaff_autotune) or default choice; else variant 0..7 */
    int32_t method;           /* chaff_method */
    int32_t precond;          /* chaff_precond: what the Pinv argument of chaff_solve holds */
    int32_t reserved;         /* must be 0 */
} chaff_solve_opts;

/* Preconditioner passed to chaff_solve as Pinv.
 *   CHAFF_PRECOND_BLOCK   [N][NB][NB] inverse self blocks from chaff_fill_Z
 *                         (the block-diagonal preconditioner of Sec. II-B);
 *   CHAFF_PRECOND_CLUSTER the buffer of chaff_cluster_precond (inverse
 *                         diagonal blocks of groups of 8 nearby wires);
 *   CHAFF_PRECOND_NBHD    the buffer of chaff_nbhd_precond (each wire's row
 *                         of the inverse of its neighbourhood's submatrix,
 *                         on Z's block pattern). */
typedef enum { CHAFF_PRECOND_BLOCK = 0, CHAFF_PRECOND_CLUSTER = 1, CHAFF_PRECOND_NBHD = 2 } chaff_precond;

/* Krylov method of each refinement cycle.  GMRES(m) with classical
 * Gram-Schmidt applied twice; COCG = conjugate-orthogonal CG, valid because
 * Z and its block-diagonal inverse are complex symmetric (bilinear a^T b),
 * with four vectors and no restart inside a cycle.  CHAFF_COCG restarts the
 * recurrence at every refinement checkpoint; CHAFF_COCG_RR keeps the search
 * direction and only replaces the recursive residual by the FP64 true one
 * (after a cycle that ended at its `restart` step cap it restarts the
 * recurrence as CHAFF_COCG does).
 * CHAFF_GCR is the generalized conjugate residual method of Sec. II-B,
 * restarted every `restart` (= m <= 200) steps and right-preconditioned:
 * it keeps the m preconditioned directions and their images under Z
 * (2m + 2 vectors), made orthonormal by classical Gram-Schmidt applied
 * twice, and minimises the residual over them at every step. */
typedef enum { CHAFF_GMRES = 0, CHAFF_COCG = 1, CHAFF_COCG_RR = 2, CHAFF_GCR = 3 } chaff_method;

typedef struct {
    int32_t cycles;           /* refinement sweeps (= GMRES restart cycles) run */
    int32_t iterations;       /* Krylov steps (one sparse product each: Arnoldi steps of
                                 GMRES, COCG or GCR steps) summed over cycles */
    double  max_rel_residual; /* final max over systems of the FP64 relative residual */
    double  seconds;          /* host wall time of the call */
} chaff_solve_stats;

size_t chaff_solve_workspace_bytes(chaff_cloud c, const chaff_solve_opts* o, int64_t n_rhs);
/*   Z        from chaff_fill_Z; Pinv the preconditioner named by o->precond
 *            (same prec; COCG needs both symmetric: they are).
 *   restart  GMRES cycle length, or the step cap of one COCG cycle.
 *   k_hat, e_hat [R][3] double: propagation direction and polarisation (unit).
 *   X        [N*NB][R] complex double, caller order; input guess if use_x0 == 1.
 *   ws       device workspace of chaff_solve_workspace_bytes.
 *   rel_res  [host out, optional] [n_clouds*R] final relative residuals (cloud-major).
 *   Host-synchronising: once per Krylov step the host reads back the count
 *   of systems still above their checkpoint (one int32), and once per cycle
 *   the FP64 residual norms. */
chaff_status chaff_solve(chaff_cloud c, const chaff_solve_opts* o, const void* Z,
                         const void* Pinv, const double* k_hat, const double* e_hat,
                         int64_t n_rhs, void* X, void* ws, size_t ws_bytes,
                         chaff_solve_stats* st, double* rel_res, chaff_stream stream);

/* ------------------------------------------------------------------ cluster preconditioner
 * The block-diagonal preconditioner of Sec. II-B taken over groups of nearby
 * wires.  Clusters are runs of CHAFF_CLUSTER_WIRES consecutive wires of one
 * cloud in the internal order (wires sorted by cloud, Morton code of their
 * neighbour-search cell, caller index); the last cluster of a cloud may be
 * shorter.  A cluster's block is the inverse, computed in FP64 with partial
 * pivoting, of the cluster's (7 w x 7 w) diagonal submatrix of Z, padded to
 * CHAFF_CLUSTER_ROWS x CHAFF_CLUSTER_ROWS with the identity.  Each block is
 * complex symmetric, as Z is, so COCG may use it.  Wires of 8 segments only
 * (CHAFF_EINVAL for a cloud built with n_seg = 20).
 *
 * Buffer M (device, 256-byte aligned, chaff_cluster_precond_bytes):
 *   [n_clusters] { int32 first wire (internal index), int32 wires }, padded
 *   to a multiple of 256 bytes, then [n_clusters][56][56] complex (prec),
 *   row-major, rows and columns in the cluster's internal wire order.
 * It is tied to the handle it was built for and to Z of the same prec. */
#define CHAFF_CLUSTER_WIRES 8
#define CHAFF_CLUSTER_ROWS 56
int64_t chaff_cluster_count(chaff_cloud c);   /* number of clusters; -1 for a NULL handle or 20 segments */
size_t chaff_cluster_precond_bytes(chaff_cloud c, chaff_prec prec);   /* 0 on a bad argument */
/* Builds M from Z (chaff_fill_Z, same prec).  Host-synchronising; returns
 * CHAFF_ESINGULAR if a cluster block has a zero pivot (M is then unusable). */
chaff_status chaff_cluster_precond(chaff_cloud c, chaff_prec prec, const void* Z, void* M,
                                   chaff_stream stream);
/* Y = M X on the internal order: X, Y [N*7][s] complex (prec), row-major,
 * distinct buffers.  Host-synchronising: M's first and last cluster entries
 * are read back and checked against the handle before any launch
 * (CHAFF_EINVAL for a buffer that is not this cloud's cluster preconditioner);
 * chaff_solve makes the same check when o->precond is CHAFF_PRECOND_CLUSTER. */
chaff_status chaff_cluster_apply(chaff_cloud c, chaff_prec prec, const void* M, const void* X,
                                 void* Y, int64_t s, chaff_stream stream);

/* ------------------------------------------------------------------ neighbourhood-inverse preconditioner
 * The block-diagonal preconditioner of Sec. II-B centred on every wire.  Wire
 * p's neighbourhood N(p) is p followed by at most size - 1 wires of its near
 * set (eq. 9), nearest first: by the FP64 squared centroid distance
 * ((dx*dx + dy*dy) + dz*dz), each operation rounded, then the lower caller
 * index.  With A_p the submatrix of Z on the wires of N(p) (their self
 * blocks and every near-pair block between them) and W_p = A_p^-1, the
 * preconditioner is
 *     M_pq = (W_p[p,q] + W_q[q,p]^T) / 2,
 * a raw block W_p[p,q] with q outside N(p) counting as zero: M is complex
 * symmetric like Z (so COCG may use it) and has blocks only on near pairs.
 * size = 1 gives the block-diagonal preconditioner; a group of mutually near
 * wires that is every member's whole neighbourhood is inverted exactly.
 * Each W_p[p, .] is computed by Gauss-Jordan elimination with partial
 * pivoting in complex FP32 (also for CHAFF_C128 buffers), so M holds FP32
 * accuracy: it changes how fast the solver converges, never the solution.
 * Wires of 8 segments only (CHAFF_EINVAL for n_seg = 20).
 *
 * Buffer M (device, 256-byte aligned, chaff_nbhd_precond_bytes):
 *   a 256-byte header {int64 tag, int64 N, int64 nnzb, int32 size, int32 prec,
 *   int32 raw (1 for the rows of chaff_nbhd_raw_rows), int32 0},
 *   then [N][size] int32 neighbourhoods (internal wire indices, slot 0 the
 *   wire itself, -1 where the near set has fewer wires) padded to a multiple
 *   of 256 bytes, then [nnzb][7][7] complex (prec): M in Z's block order
 *   (zero blocks where neither wire is in the other's neighbourhood).
 * It is tied to the handle it was built for and to Z of the same prec. */
#define CHAFF_NBHD_MAX 8
size_t chaff_nbhd_precond_bytes(chaff_cloud c, chaff_prec prec, int32_t size);   /* 0 on a bad argument */
/* Builds M from Z (chaff_fill_Z, same prec); 1 <= size <= CHAFF_NBHD_MAX.
 * Host-synchronising; returns CHAFF_ESINGULAR if a neighbourhood system has a
 * zero pivot (M is then unusable).  chaff_solve reads M's header back and
 * checks it against the handle and prec when o->precond is CHAFF_PRECOND_NBHD
 * (CHAFF_EINVAL for another buffer). */
chaff_status chaff_nbhd_precond(chaff_cloud c, chaff_prec prec, int32_t size, const void* Z, void* M,
                                chaff_stream stream);
/* The same build without the symmetrisation: M's blocks hold the raw rows
 * W_p[p,q] at the positions (p, q), q in N(p), and zero elsewhere; the header
 * is tagged raw and chaff_solve refuses the buffer.  The training targets of
 * the learned form below. */
chaff_status chaff_nbhd_raw_rows(chaff_cloud c, chaff_prec prec, int32_t size, const void* Z, void* M,
                                 chaff_stream stream);

/* ------------------------------------------------------------------ learned neighbourhood inverse
 * Growth part (4), the block-preconditioner form: the network of the learned
 * guess (CHAFF_MLP_NFEAT inputs, three SiLU layers, CHAFF_MLP_NOUT outputs;
 * parameters theta as for chaff_mlp_forward) predicts the raw rows of the
 * neighbourhood-inverse preconditioner from the neighbourhood's geometry,
 * and the predicted rows are symmetrised like the computed ones.  Samples
 * are (wire i, slot s, column c), row (i size + s) 7 + c in the internal wire
 * order: slot s of i's neighbourhood (q = N(i)[s]), column c of the block.
 * Each wire gets a canonical tangent tau = sigma t, sigma = +1 when the first
 * nonzero of (t_z, t_y, t_x) is positive, else -1; S = sigma P maps rooftop
 * coefficients to the canonical frame (P reverses the 7 rooftops when
 * sigma = -1), and a block W becomes S_i W S_q there.
 *   features (BF16, FP64 values rounded once; d_xy = c_y - c_x,
 *   E(x) = exp(-j 2 pi x / lambda), all zero for an empty slot):
 *     [c] = 1, [7 + s] = 1 (one-hot column and slot);
 *     [15], [16] = 10 (L_i/lambda - 1/2), 10 (L_q/lambda - 1/2);
 *     [17..22] = |d_iq|/d_c, tau_i.d_iq/d_c, tau_q.d_iq/d_c, tau_i.tau_q, Re, Im E(|d_iq|);
 *     [23] = |N(i)| / 8;
 *     member t of N(i) at 24 + 15 t: 1, 10 (L_t/lambda - 1/2), the six pair
 *     numbers of (i, t), the six of (q, t), 1 if t = q or t and q are near;
 *     [144..191] = 0.
 *   targets: y[2r] + j y[2r+1] = 0.05 (S_i (W_i[i,q] - delta_iq Pinv_i) S_q)[r][c]
 *   (FP32): the departure from the block-diagonal preconditioner (Pinv the
 *   inverse self blocks of chaff_fill_Z), so that zero outputs give it exactly.
 * Wires of 8 segments and finite d_c only. */
/* feat [n_rows][CHAFF_MLP_NFEAT] BF16 for rows [row0, row0 + n_rows) of the
 * neighbourhoods stored in M (any buffer of chaff_nbhd_precond / _raw_rows;
 * its header is read back: host-synchronising). */
chaff_status chaff_nbhd_mlp_features(chaff_cloud c, const void* M, int64_t row0, int64_t n_rows,
                                     uint16_t* feat, chaff_stream stream);
/* Y [N size 7][CHAFF_MLP_NOUT] FP32 targets from a buffer of chaff_nbhd_raw_rows
 * and the inverse self blocks Pinv [N][7][7] of chaff_fill_Z (same prec;
 * host-synchronising header check). */
chaff_status chaff_nbhd_mlp_targets(chaff_cloud c, chaff_prec prec, const void* M, const void* Pinv,
                                    float* Y, chaff_stream stream);
size_t chaff_nbhd_mlp_workspace_bytes(chaff_cloud c, int32_t size);   /* 0 on a bad argument */
/* Builds the learned preconditioner into M (chaff_nbhd_precond_bytes, 256-byte
 * aligned): neighbourhoods, features, the network in chunks, raw rows from its
 * outputs, symmetrisation.  The result is a CHAFF_PRECOND_NBHD buffer.
 * ws: device workspace of chaff_nbhd_mlp_workspace_bytes.  Host-synchronising. */
chaff_status chaff_nbhd_mlp_precond(chaff_cloud c, chaff_prec prec, int32_t size, const float* theta,
                                    const void* Pinv, void* M, void* ws, size_t ws_bytes,
                                    chaff_stream stream);

/* Excitation alone: U [N*NB][R] complex double (caller order), eq. (4) without
 * its -(j/(w mu0)) factor, closed-form triangle transform. */
chaff_status chaff_excitation(chaff_cloud c, const double* k_hat, const double* e_hat,
                              int64_t n_rhs, void* U, chaff_stream stream);

/* Block-sparse product Y = Z X on the internal order (the matvec of the
 * Krylov solver, complexity O(b_mean N) of Sec. II-B).
 *   X, Y [N*NB][s] complex (prec), internal order, row-major.
 *   variant -1 = the tuned/heuristic choice. */
chaff_status chaff_spmm(chaff_cloud c, chaff_prec prec, const void* Z, const void* X,
                        void* Y, int64_t s, int32_t variant, chaff_stream stream);

/* ------------------------------------------------------------------ autotuning
 * chaff_autotune times every block-sparse product variant (0: one output row
 * per lane; 1: RHS tile per wave; 2: half-width tile; 3: tile in XCD-aware
 * workgroup order; 4: XCD-aware half-width tile; 5: one lane per output row
 * accumulating up to 16 RHS columns, every Z row loaded once; 6: one wave per
 * block row (4, 2 and 4 rows per wave at 4, 8 and 16 columns), the blocks
 * staged in LDS; 7: 6 in XCD-aware order) for this cloud, precision
 * and RHS count on the caller's Z and two [N*NB][s] buffers (contents of Y are
 * overwritten, X is read), and records the fastest in a process-wide table
 * keyed by (N, nnzb, s, prec).  Every later call with variant -1 (chaff_spmm,
 * and the products inside chaff_solve, including the COCG product's tile
 * width and workgroup order) uses the recorded choice.
 *   best_variant, best_ms [host out, optional].  Synchronises `stream`.
 * chaff_tune_report writes the table as JSON text into buf [host] (at most len
 * bytes, NUL-terminated) and returns the length needed including the NUL. */
chaff_status chaff_autotune(chaff_cloud c, chaff_prec prec, const void* Z, void* X, void* Y, int64_t s,
                            int32_t* best_variant, double* best_ms, chaff_stream stream);
int32_t chaff_tune_report(char* buf, int32_t len);

/* ------------------------------------------------------------------ rcs
 * Far field of the currents X (caller order, complex double [N*NB][R]):
 * S = sum_n w_n(r_hat, e) x_n with w_n = int L_n (t_n . e) exp(+j k r_hat . r) ds,
 * sigma = |S|^2/(4 pi) [m^2], summed separately over each cloud.
 *   monostatic = 1: M == R, observation m pairs with RHS m;
 *                   sigma [n_clouds][R].
 *   monostatic = 0: every (RHS, direction); sigma [n_clouds][R][M].
 *   obs_dir, obs_pol [M][3] double (unit; pol transverse to dir).
 *   ws: device workspace of chaff_rcs_workspace_bytes. */
size_t chaff_rcs_workspace_bytes(chaff_cloud c, int64_t n_rhs, int64_t n_dirs, int32_t monostatic);
chaff_status chaff_rcs(chaff_cloud c, const void* X, int64_t n_rhs, const double* obs_dir,
                       const double* obs_pol, int64_t n_dirs, int32_t monostatic,
                       double* sigma, void* ws, size_t ws_bytes, chaff_stream stream);

/* ------------------------------------------------------------------ rcs without a workspace
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc): chaff_rcs with
 * the same arguments and results but no workspace.  Its scratch (chunk bounds
 * and per-chunk partial sums, chaff_rcs_workspace_bytes of them) lives in a
 * fixed device array of CHAFF_RCS_SCRATCH_BYTES inside the library, one copy
 * per GPU, held until the process ends; the call allocates nothing.  It runs
 * on the current device (the stream must belong to it) and synchronises the
 * stream before returning, as chaff_rcs does.
 * Returns CHAFF_EWORKSPACE if chaff_rcs_workspace_bytes(c, n_rhs, n_dirs,
 * monostatic) exceeds CHAFF_RCS_SCRATCH_BYTES (then use chaff_rcs).
 * Every call on one GPU uses that GPU's one array: calls that overlap in time
 * on one GPU (several host threads or streams) race and must be serialised by
 * the caller. */
#define CHAFF_RCS_SCRATCH_BYTES (64u << 20)
chaff_status chaff_rcs_noalloc(chaff_cloud c, const void* X, int64_t n_rhs, const double* obs_dir,
                               const double* obs_pol, int64_t n_dirs, int32_t monostatic, double* sigma,
                               chaff_stream stream);

/* ------------------------------------------------------------------ learned initial guess
 * Not part of the paper's method.  A small network predicts, for each wire p
 * and incidence r, the wire's 7 currents from its neighbourhood; the result
 * is the initial iterate of chaff_solve (use_x0 = 1).  The solver still
 * drives the true residual of the S-NFC system to the requested tolerance,
 * so the guess changes the iteration count, never the solution.
 *
 * Samples (rows): row = p*R + r, p in caller order.
 * Canonical frame: s_p = +1 if t_p . e_r >= 0 else -1, tau_p = s_p t_p.
 * Reversing a wire reverses its rooftop order and negates the coefficients,
 * so the canonical currents are x~_{p,q} = s_p x_{p,q'}, q' = q if s_p = 1
 * else 6 - q.  With k = 2 pi/wavelength, D_p = L_p/8, beta_p = k k_hat.tau_p,
 * s_q = -L_p/2 + (q+1) D_p and sinc x = sin x / x, the 192 features of a row
 * are
 *   [0]        10 (L_p/wavelength - 1/2)
 *   [1]        n_p/16, n_p = other wires of the cloud within d_c
 *   [2+2q, 3+2q]  Re, Im of (tau_p.e) sinc^2(beta_p D_p/2) exp(-j beta_p s_q)
 *              (the excitation of eq. (4) in the canonical frame, divided by
 *              D_p, incident phase at c_p removed), q = 0..6
 *   [16+11j .. 26+11j]  for the j-th nearest other wire p' within d_c
 *              (ascending squared distance as in the near-set test, ties by
 *              caller index; j < 16), d = c_p' - c_p:
 *              |d|/d_c, tau_p.d/d_c, tau_p'.d/d_c, tau_p.tau_p',
 *              Re, Im of (tau_p'.e) exp(-j k k_hat.d),
 *              10 (L_p'/wavelength - 1/2), k_hat.tau_p',
 *              Re, Im of exp(-j k |d|), 1;  zeros if empty.
 * Features are evaluated in FP64 and stored as BF16 bit patterns (uint16),
 * rounded FP64 -> FP32 -> BF16, each step to nearest even.
 *
 * Network: 192 -> 128 -> 128 -> 128 -> 14, SiLU after the hidden layers.
 * theta [CHAFF_MLP_NPARAM] float: W1 [192][128], b1 [128], W2 [128][128],
 * b2, W3 [128][128], b3, W4 [128][14], b4 [14]; W[i][o] input-major.
 * Products take BF16 weights and BF16 layer inputs with FP32 accumulation;
 * biases, pre-activations and SiLU are FP32.
 * Outputs / targets [rows][14] float: the departure of the currents from the
 * wire's isolated response b_p = Pinv_p u_p (the block-Jacobi solution:
 * Pinv_p the inverse self block of chaff_fill_Z, u_p the wire's excitation),
 *   y[2q] + j y[2q+1] = (x~_{p,q} - b~_{p,q}) exp(+j k k_hat.c_p) / 0.5,
 * b~ the canonical form of b.
 * Loss: mean over rows and the 14 outputs of (y - t)^2.
 * Buffers must be 16-byte aligned.  Requires a finite d_c > 0 and wires of
 * 8 segments. */
#define CHAFF_MLP_K 16
#define CHAFF_MLP_NFEAT 192
#define CHAFF_MLP_HIDDEN 128
#define CHAFF_MLP_NOUT 14
#define CHAFF_MLP_NPARAM 59534

/* Features of rows [row0, row0 + n_rows) into feat [n_rows][192] (uint16 BF16). */
chaff_status chaff_mlp_features(chaff_cloud c, const double* k_hat, const double* e_hat, int64_t n_rhs,
                                int64_t row0, int64_t n_rows, uint16_t* feat, chaff_stream stream);

/* Targets Y [N*R][14] float from currents X [N*7][R] complex double (caller
 * order); Pinv [N][7][7] complex (prec) from chaff_fill_Z. */
chaff_status chaff_mlp_targets(chaff_cloud c, chaff_prec prec, const void* Pinv, const double* k_hat,
                               const double* e_hat, int64_t n_rhs, const void* X, float* Y,
                               chaff_stream stream);

/* Workspace of chaff_mlp_forward (train = 0) or chaff_mlp_grad / chaff_mlp_train_step
 * (train = 1) for n_rows rows. */
size_t chaff_mlp_workspace_bytes(int64_t n_rows, int32_t train);

/* Network outputs Y [n_rows][14] of feat [n_rows][192]. */
chaff_status chaff_mlp_forward(const float* theta, const uint16_t* feat, int64_t n_rows, float* Y,
                               void* ws, size_t ws_bytes, chaff_stream stream);

/* Loss and gradient over the rows idx[0..n_rows) of feat and T (idx NULL: rows
 * 0..n_rows-1).  grad [CHAFF_MLP_NPARAM] float, loss [1] float (device; may be
 * NULL).  Deterministic: every sum runs in a fixed order. */
chaff_status chaff_mlp_grad(const float* theta, const uint16_t* feat, const float* T, const int64_t* idx,
                            int64_t n_rows, float* grad, float* loss, void* ws, size_t ws_bytes,
                            chaff_stream stream);

/* One Adam step on theta with moments m, v (float [CHAFF_MLP_NPARAM]); step t >= 1. */
chaff_status chaff_mlp_adam(float* theta, float* m, float* v, const float* grad, int32_t t, float lr,
                            float beta1, float beta2, float eps, chaff_stream stream);

/* chaff_mlp_grad followed by chaff_mlp_adam (gradient kept in the workspace). */
chaff_status chaff_mlp_train_step(float* theta, float* m, float* v, int32_t t, float lr, float beta1,
                                  float beta2, float eps, const uint16_t* feat, const float* T,
                                  const int64_t* idx, int64_t n_rows, float* loss, void* ws,
                                  size_t ws_bytes, chaff_stream stream);

/* Initial guess X [N*7][R] complex double (caller order) for chaff_solve with
 * use_x0 = 1: features, network and the inverse of the target map (isolated
 * response from Pinv plus the predicted departure), in chunks of at most
 * 2^18 rows. */
size_t chaff_mlp_guess_workspace_bytes(chaff_cloud c, int64_t n_rhs);
chaff_status chaff_mlp_guess(chaff_cloud c, chaff_prec prec, const void* Pinv, const float* theta,
                             const double* k_hat, const double* e_hat, int64_t n_rhs, void* X, void* ws,
                             size_t ws_bytes, chaff_stream stream);

/* ------------------------------------------------------------------ profiling
 * Per-kernel timing of the library's own launches with HIP events recorded
 * on the launch stream (used for roofline figures).  chaff_profile_enable(1)
 * clears the record and starts; (0) stops.  chaff_profile_read waits for the
 * recorded events and writes one aggregate per kernel name (at most max_out)
 * into out [host]; returns the number written. */
typedef struct {
    char    name[48];
    int64_t launches;
    double  total_ms, min_ms, max_ms;
    double  bytes;            /* algorithmic HBM bytes summed over launches (0: not stated) */
    double  flops;            /* algorithmic flops summed over launches (0: not stated) */
} chaff_kernel_time;
chaff_status chaff_profile_enable(int32_t on);
int32_t chaff_profile_read(chaff_kernel_time* out, int32_t max_out);

/* ------------------------------------------------------------------ misc */
/* The product-variant tuning table as JSON, written to / merged from a file
 * (entries keyed by unknowns per wire, wires, stored blocks, RHS count and
 * precision; a loaded entry replaces a recorded one with the same key).
 * chaff_tune_load: n_entries [host out, optional] entries read; CHAFF_EINVAL
 * if the file cannot be read or is not such a table (nothing is changed). */
chaff_status chaff_tune_save(const char* path);
chaff_status chaff_tune_load(const char* path, int32_t* n_entries);

void chaff_destroy(chaff_cloud c);
const char* chaff_last_error(void);
const char* chaff_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CHAFF_H */
