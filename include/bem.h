/*
 * bem.h -- C-ABI of libbem, the MI355X (gfx950) hot path of the 3D-ACA / H-matrix
 * accelerated Laplace-domain boundary element method for 3D elastodynamics
 * (Keshava & Schanz, "A 3D-ACA accelerated time domain boundary element method for
 * elastodynamics using FMM and H-matrix techniques").
 *
 * What the library computes
 *   Collocation BEM with flat triangles (Sec. 2.3, eq. (tri)), piecewise-constant trial
 *   functions and collocation at element centroids (Sec. 2.3), for the Laplace-domain
 *   single layer V and double layer K (eqs. (SLP), (DLP), (discrVK) with U* replaced by
 *   its Laplace transform U(y - x, s), Sec. 2.4) at the complex frequencies s_l of the
 *   gCQ contour.  The three-dimensional array of 3x3 blocks ENTRY(i, j, l) (Sec. 2.4,
 *   "M x M x N_Q") is either assembled densely or compressed with the matrix-valued
 *   3D-ACA of Algorithm 1 (Sec. 3) on the blocks of an H-matrix partition (Sec. 3.1,
 *   eqs. (cluster), (adm)), far-field faces being approximated per slice by matrix-valued
 *   ACA with QR/SVD recompression (eq. (ACA)).  Products apply the compressed array at
 *   every frequency (the face-fibre form of eq. (3DacaMult)).
 *
 * Conventions (all entry points)
 *   - Every function returns int: BEM_OK (0) on success, a negative BEM_ERR_* code on
 *     failure, a positive BEM_WARN_* code for success with a warning.  On failure no
 *     output buffer is guaranteed to be written; bem_last_error() gives a message.
 *   - Complex numbers are interleaved (re, im) pairs of double (complex128) or float
 *     (complex64), compatible with C99 _Complex and numpy/torch complex layouts.
 *   - Indices are 0-based.  DOF index = 3 * element + component.  The ABI always speaks
 *     mesh order; the cluster permutation is internal.
 *   - Triangle orientation: the unit normal is (v1 - v0) x (v2 - v0) normalised and must
 *     point out of the domain Omega (into the exterior for a bounded body, into the
 *     cavity for an exterior problem).
 *   - Buffers: BEM_DEVICE_PTR in `flags` means the pointers are device pointers on the
 *     context's device (e.g. torch tensor data_ptr()); otherwise they are host pointers
 *     and the library stages them through device memory.  Work is issued on the stream
 *     set by bem_set_stream (default: the null stream); calls with host buffers return
 *     after the results are in the host buffer; calls with device buffers return after
 *     enqueueing (synchronise the stream before reading).
 *   - Inputs are copied; the caller keeps ownership of everything it passes.  Opaque
 *     objects (bem_ctx, bem_op) are owned by the library and released by *_destroy.
 *   - A context is not thread-safe; distinct contexts are independent.  No C++
 *     exception crosses this interface.
 */
#ifndef BEM_H
#define BEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_ctx bem_ctx;
typedef struct bem_op bem_op;

/* return codes */
#define BEM_OK 0
#define BEM_ERR_ARG (-1)       /* invalid argument (null pointer, size, enum value) */
#define BEM_ERR_MESH (-2)      /* node index out of range, degenerate triangle, K < 1 */
#define BEM_ERR_MATERIAL (-3)  /* rho <= 0, cs <= 0 or cp <= cs, non-finite values */
#define BEM_ERR_FREQ (-4)      /* Re s <= 0, non-finite, L < 1 */
#define BEM_ERR_STATE (-5)     /* mesh, material or frequencies not set yet */
#define BEM_ERR_HIP (-6)       /* a HIP runtime call failed */
#define BEM_ERR_NOMEM (-7)     /* device allocation failed or the compression pool overflowed */
#define BEM_ERR_NODEVICE (-8)  /* GPU call on a host-only context (device = -1) */
#define BEM_WARN_BULK 1        /* cp^2 < 4/3 cs^2: negative bulk modulus (still computed) */
#define BEM_WARN_NOCONV 2      /* bem_solve: tolerance not met within max_iter / max_refine */

/* operators */
#define BEM_OP_V 0     /* single layer V (eq. (SLP)), kernel U */
#define BEM_OP_K 1     /* double layer K (eq. (DLP)), kernel T, Cauchy principal value */
#define BEM_OP_HK 2    /* C + K with the free term C = I/2 at smooth points (eq. (SBIE)) */
#define BEM_OP_TABLE 3 /* ENTRY read from a user table (bem_set_entry_table); for tests */
#define BEM_OP_KL0 4   /* bem_entries only: the double layer against the hat function of vertex 0 */
#define BEM_OP_KL1 5   /* (1, 2) of element j: int_{gamma_j} T(x_i, y) lambda_v(y) dy, the element */
#define BEM_OP_KL2 6   /* share of the continuous piecewise-linear basis of eqs. (subspace), (basis) */

/* precision of entry generation and storage */
#define BEM_PREC_F64 0   /* complex128 everywhere */
#define BEM_PREC_MIXED 1 /* far field complex64 (entries, factors, products); near field,
                            singular/near-singular quadrature, pivots and norms complex128 */

/* flags */
#define BEM_DEVICE_PTR 1   /* buffers are device pointers */
#define BEM_SHARED_X 2     /* bem_apply: x has shape [nrhs][3K], the same for every frequency */
#define BEM_TRANSPOSE 4    /* bem_apply, bem_solve: the plain transpose A(s_l)^T (no conjugation);
                              the adjoint of a solution needs A^T solves */
#define BEM_FREE_TERM 8    /* bem_apply_linear_dl: add the free term C = I/2 (C + K) */

/* Quadrature options (Sec. 2.3: Duffy for the singular collocation integrals; the rest is
 * this library's documented reading).  regular pairs: 7-point degree-5 rule; near pairs
 * (near_on): the same rule on 4^2 sub-triangles if |x_i - c_j| < near_r1 * lmax_j, on 4^1
 * if < near_r2 * lmax_j (lmax_j = longest edge of element j); self pairs: polar Duffy
 * about the centroid on 3 sub-triangles with self_nt x self_nr Gauss-Legendre points
 * (principal value for K, with the leading 1/rho^2 part integrated analytically). */
typedef struct {
    int32_t near_on;     /* default 0 */
    double near_r1;      /* default 1.5 */
    double near_r2;      /* default 3.0 */
    int32_t self_nt;     /* default 8, 1..16 */
    int32_t self_nr;     /* default 8, 1..16 */
} bem_quad;

/* Options of bem_compress (Sec. 3, Sec. 3.1, Table 2). */
typedef struct {
    double eps3d;        /* 3D-ACA tolerance epsilon of eq. (precision) */
    double eps_aca;      /* per-slice ACA tolerance; <= 0 selects eps3d / 100 (Sec. 4.1) */
    double eta;          /* admissibility parameter of eq. (adm); default 1.5 */
    int32_t leaf;        /* b_min: largest leaf cluster (elements); default 64 */
    int32_t prec;        /* BEM_PREC_F64 or BEM_PREC_MIXED */
    double mixed_eps_floor; /* MIXED only: far-field tolerances are raised to at least this
                               value (complex64 entries cannot resolve less); default 1e-5 */
    int64_t pool_bytes;  /* working pool of the faces, fibres and factors of one block group
                            (bytes; 0 = auto: 60 % of the free memory, grown on demand).
                            The blocks are compressed in consecutive groups whose faces of
                            min(L, 32) steps fit the pool; each group is compacted into a
                            pool of exact size before the next starts */
    int32_t far_dense_max; /* admissible blocks whose smaller side has at most this many
                              elements keep dense faces (their per-slice ACA rank is close to
                              full); 0 = per-slice ACA on every admissible block; default 48 */
    int32_t aca_rounds;   /* per-slice ACA runs that reach the column capacity of the pass (96
                             columns) on a face whose factors could still save memory: 0 = the
                             face stays dense (default); > 0 = the columns are recompressed
                             (eq. (ACA), at a quarter of the face tolerance) and the ACA resumes
                             from them, up to this many times per pass.  For memory-bound
                             compressions: it trades recompression time for storage */
    int32_t face_order;   /* where the per-slice ACA of the admissible blocks' faces runs:
                             BEM_FACES_AFTER (default): a pass over the exact faces once the
                             3D-ACA of every block has ended (faces compressed to an absolute
                             tolerance eps_aca ||C|| / ||f_d||);
                             BEM_FACES_IN_LOOP: the paper's order (Sec. 3.1, the H-matrix
                             ACA): in every step the residual face is approximated by the ACA
                             and recompressed (eq. (ACA)) relative to its own norm (stop when
                             ||U_k|| ||V_k|| <= eps_aca ||U V^H||, truncation at eps_aca of the
                             singular values), the pivot of Algorithm 1 is searched on the
                             reconstruction of the factors, and the reconstruction is the face
                             that the later residuals, the fibre and the norm of eq. (FrobNorm)
                             use.  A face whose ACA does not resolve within 96 columns, or whose
                             factors would not take less memory, stays exact.  aca_rounds does
                             not apply */
} bem_aca_opts;
#define BEM_FACES_AFTER 0
#define BEM_FACES_IN_LOOP 1

/* Statistics of an operator (compression rate as defined in Sec. 4.1: memory of the
 * compressed representation over the memory of the dense M x M x L array). */
typedef struct {
    int64_t n_blocks, n_near, n_far, n_dense_fallback;
    int32_t rank_min, rank_max;   /* 3D-ACA ranks r_b over blocks (Fig. 5 reports these) */
    double rank_mean;
    int32_t aca_rank_max;         /* largest rank kk of a far face stored as factors */
    double aca_rank_mean;         /* mean kk over the far faces stored as factors */
    int64_t bytes;                /* device bytes of faces, factors and fibres */
    double compression_rate;      /* bytes / (L * (3K)^2 * 16), with several components the
                                     sum of L (3K_c)^2 16 over the components */
    int64_t entries_generated;    /* ENTRY(i, j, l) 3x3 blocks evaluated during compression */
    int64_t n_far_faces;          /* far faces stored as factors */
    double seconds;               /* wall time of the compression call */
    double kernel_ms;             /* device time of the compression (HIP events on the context
                                     stream from the first to the last launch) */
    int64_t n_aca_dense;          /* far faces of ACA blocks kept dense: the per-slice ACA did
                                     not resolve them within its column cap, or the factors
                                     would not take less memory than the face */
    double aca_cols_mean;         /* ACA columns before recompression, mean over the faces
                                     stored as factors */
    double aca_ms;                /* device time of the per-slice ACA + recompression pass */
    double face_ms;               /* device time of the face kernels of the 3D-ACA steps (HIP
                                     events around each step's face launches) */
    int64_t face_launches;        /* face kernel launches */
    int64_t face_pairs;           /* (i, j) pairs generated by the face kernels */
    double face_flop;             /* algorithmic flops of the face kernels: per pair of step d,
                                     7 regular-rule kernel evaluations (125 flops for U, 236 for
                                     T) and d residual updates (216 flops) */
    double recomp_ms;             /* device time of the recompression kernel (k_face_recomp) */
    int64_t recomp_launches;      /* its launches */
    double recomp_flop;           /* algorithmic flops of the recompressions (complex
                                     multiply-add = 8): Grams, Choleskys, core product, pivoted
                                     QR, Jacobi sweeps, coefficients, reflectors,
                                     back-substitutions and output products, as executed */
    int64_t entries_regular;      /* entries_generated split by rule: the pairs of the kept */
    int64_t entries_near;         /* faces by class (regular 7-point, near subdivision, self */
    int64_t entries_self;         /* polar rule), and the rest (fibres and pivot entries) in */
    int64_t entries_other;        /* entries_other */
    double face_bytes;            /* algorithmic HBM bytes of the face kernels: per pair of step
                                     d, the new face block written and the d earlier face
                                     blocks read (72 B each in complex64, 144 B in complex128) */
    int64_t block_groups;         /* groups the blocks were compressed in, one after the other
                                     (1 unless the faces of all blocks would not fit the memory
                                     or bem_aca_opts.pool_bytes) */
    double apply_macs_c64;        /* algorithmic work of bem_apply: complex multiply-adds per
                                     column (right-hand side and frequency) of the faces and
                                     factors stored in complex64 (9 m n per dense face,
                                     3 (m + n) kk per factored one) */
    double apply_macs_c128;       /* the same for the faces and factors stored in complex128 */
    double apply_macs_sel;        /* the same per right-hand side for the dense-fallback faces
                                     (each acts at one frequency) */
    double apply_macs_fibre;      /* complex multiply-adds per column of the fibres (9 n per face) */
    double aca_kernel_ms;         /* device time of the per-slice ACA kernel (k_face_aca), HIP
                                     events around each launch */
    int64_t aca_launches;         /* its launches */
    double aca_flop;              /* its algorithmic flops: per rank-3 step t of a face, the
                                     residual 3-row and 3-column blocks updated by the 3t earlier
                                     columns (9 (m + n) 3t complex multiply-adds) and the pivot
                                     inverse applied (27 m) */
    double aca_bytes;             /* its algorithmic bytes: per step the 3 (m + n) 3t earlier
                                     column entries read (FP64), 9 (m + n) face entries read and
                                     9 (m + n) column entries written */
} bem_stats;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device`; device = -1 gives a host-only context (mesh,
 * material, frequency validation and partition queries; GPU calls return
 * BEM_ERR_NODEVICE).  *out is set to NULL on failure. */
int bem_create(bem_ctx **out, int32_t device);
/* Releases the context and all its device memory (operators must be destroyed first). */
int bem_destroy(bem_ctx *ctx);
/* Message of the last error on this context (never NULL; empty when none). */
const char *bem_last_error(const bem_ctx *ctx);
/* HIP stream (hipStream_t as void*) for all subsequent work of this context. */
int bem_set_stream(bem_ctx *ctx, void *hip_stream);

/* Flat triangle mesh Gamma^h = union of K triangles (Sec. 2.3, eq. (tri)).
 * nodes: [n_nodes][3] double (host), tris: [K][3] int32 (host).
 * Errors: BEM_ERR_MESH for K < 1, an index outside [0, n_nodes) or a zero-area triangle. */
int bem_set_mesh(bem_ctx *ctx, const double *nodes, int64_t n_nodes, const int32_t *tris, int64_t K);

/* Several meshes in one context (the meshes of a batch sharing material and contour points):
 * comp[e] in [0, ncomp) names the mesh of element e (every component non-empty); the
 * elements of different components do not interact.  bem_compress then partitions each
 * component apart (no block couples two components) and compresses all of them in one set of
 * launches, and the products of the operator are those of every mesh at once (block
 * diagonal).  bem_entries ignores components; bem_assemble_dense, bem_apply_mf and
 * bem_adjoint_v return BEM_ERR_STATE on a context of several components.  comp = NULL or
 * ncomp <= 1 restores one component; bem_set_mesh resets to one component.  Host array,
 * copied.  Errors: BEM_ERR_STATE before bem_set_mesh, BEM_ERR_ARG for an index out of range or
 * an empty component. */
int bem_set_components(bem_ctx *ctx, const int32_t *comp, int32_t ncomp);

/* Material (Sec. 2.1, eq. (lame)): density rho, compression and shear wave speeds
 * cp = c1 > cs = c2 > 0.  Returns BEM_WARN_BULK if cp^2 < 4/3 cs^2. */
int bem_set_material(bem_ctx *ctx, double rho, double cp, double cs);

/* Contour points s_l, l = 0..L-1 (Sec. 2.4, eq. (laptrans): Re s > 0), [L][2] double host.
 * Conjugate pairs (Sec. 4.1) are allowed and detected (see bem_freq_pairs). */
int bem_set_frequencies(bem_ctx *ctx, const double *s, int32_t L);
/* Number of l with s_l = conj(s_m) for some m != l (diagnostic). */
int bem_freq_pairs(const bem_ctx *ctx, int32_t *n_pairs);

/* Quadrature options; NULL restores the defaults. */
int bem_set_quadrature(bem_ctx *ctx, const bem_quad *q);

/* Table source for BEM_OP_TABLE: ENTRY(i, j, l) = table[((l * K + i) * K + j)][3][3]
 * complex128, device pointer, valid until replaced; the context does not own it.  Used by
 * tests to run the compression on synthetic tensors of known rank. */
int bem_set_entry_table(bem_ctx *ctx, const void *table_dev);

/* ---------------------------------------------------------------- generators */

/* Raw generator (Sec. 2.3 eq. (discrVK) at s_l; Algorithm 1's ENTRY):
 * out[e] = ENTRY(op, i[e], j[e], l[e]) as [n][3][3] complex (row = load direction /
 * collocation component, column = trial component).  prec: BEM_PREC_F64 gives complex128
 * output; BEM_PREC_MIXED gives complex128 output whose regular pairs were computed in
 * float (near and self pairs stay FP64).  i, j, l, out: host or device per flags.
 * n = 0 is a no-op.  Errors: BEM_ERR_ARG for an index out of range (checked on the host
 * for host buffers, by the kernel for device buffers: offending entries are then NaN). */
int bem_entries(bem_ctx *ctx, int32_t op, int32_t prec, int64_t n, const int32_t *i, const int32_t *j,
                const int32_t *l, void *out, int32_t flags);

/* Dense assembly of all L slices (the uncompressed array of Sec. 2.4), complex128,
 * layout [L][3K][3K] row-major, kept on the device inside *out. */
int bem_assemble_dense(bem_ctx *ctx, int32_t op, int32_t prec, bem_op **out);

/* Copies the dense slices of an operator made by bem_assemble_dense to `dst`
 * ([L][3K][3K] complex128, host or device per flags). */
int bem_op_dense_copy(const bem_op *op, void *dst, int32_t flags);

/* Compression (Sec. 3, Algorithm 1 with matrix-valued pivots, eq. (SVD); Sec. 3.1):
 * PCA cluster tree with leaf size opts->leaf, admissibility eq. (adm) with opts->eta,
 * 3D-ACA on every block over exact dense residual faces, then per-slice ACA +
 * recompression (eq. (ACA)) of every face of the admissible blocks whose smaller side
 * exceeds opts->far_dense_max, to the absolute tolerance eps_aca ||C^(r)||_F / ||f_d||_F
 * (each face-fibre term errs by at most about eps_aca ||C^(r)||_F); a face stays dense when
 * its ACA does not resolve it within the column cap or its factors would not save memory.
 * Dense fallback when no regular pivot exists (Algorithm 1's "sigma_3 = 0 for all pairs",
 * taken as sigma_3 <= 1e-12 x the largest 3x3 block of the slices formed so far).
 * opts may be NULL (eps3d = 1e-6, eps_aca = eps3d / 100, eta = 1.5, leaf = 64, F64). */
int bem_compress(bem_ctx *ctx, int32_t op, const bem_aca_opts *opts, bem_op **out);

/* The per-slice ACA + recompression (Sec. 3.1, eq. (ACA)) that bem_compress applies to a
 * far face, run on one given matrix (for tests).  A: [3m][3n] row-major host matrix of m x n
 * 3x3 blocks, complex128 (prec BEM_PREC_F64) or complex64 (BEM_PREC_MIXED); copied.
 * tol: absolute tolerance of the ACA stop test (||U_k||_F ||V_k||_F <= tol for the newest
 * 3 columns) and of the truncation (dropped singular values: sqrt(sum s^2) <= tol).
 * max_cols: ACA column cap (multiple of 3 after rounding down; <= 0 selects the library's
 * cap 3 ceil(2 m n / (m + n))); at most 3 min(m, n) and 192.
 * Out: *kc = ACA columns, -1 when the ACA did not resolve the matrix (it would stay dense);
 * *kk = rank of the factors, 0 when they would not take less memory than the matrix.
 * U ([3m][kk]) and V ([3n][kk]), row-major host buffers of the precision of A holding at
 * least 9 m min(m, n) and 9 n min(m, n) entries, receive Ubar and Vbar with
 * A ~= Ubar Vbar^H when kk > 0 (either may be NULL).
 * Errors: BEM_ERR_ARG for m, n < 1, m * n > 2^22, bad prec, tol < 0 or A NULL. */
int bem_aca_matrix(bem_ctx *ctx, int32_t prec, int32_t m, int32_t n, const void *A, double tol, int32_t max_cols,
                   int32_t *kc, int32_t *kk, void *U, void *V);

/* The computation of bem_aca_matrix on device buffers with no allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no hipMalloc, hipFree or allocating library call is made.  The working copy of
 * A, the ACA columns and the recompression matrices live in one library-held device array of
 * BEM_ACA_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends; its address is looked
 * up in bem_create, or on the first call on a device).  Every call on one GPU shares that
 * array and leaves the last call's contents in it: calls that overlap on one GPU (several
 * streams or threads) race.
 *   A: device [3m][3n] row-major, complex128 (BEM_PREC_F64) or complex64 (BEM_PREC_MIXED),
 *   read only.  tol, max_cols: as bem_aca_matrix.  kc_kk: device int32[2] receives (kc, kk)
 *   as bem_aca_matrix defines them.  U, V: device buffers of A's precision with room for
 *   9 m min(m, n) and 9 n min(m, n) entries; when kk > 0 they receive Ubar ([3m][kk]) and
 *   Vbar ([3n][kk]) row-major, A ~= Ubar Vbar^H; otherwise they are not written.  All
 *   pointers must be device memory of the context's device, aligned to their element size.
 *   Work is enqueued on the context's stream; the call returns without waiting.
 * Errors: BEM_ERR_ARG for m or n outside [1, BEM_ACA_NOALLOC_MAX_ELEMENTS], bad prec, tol < 0,
 * NULL, host or misaligned pointers; BEM_ERR_HIP when the scratch address cannot be found. */
#define BEM_ACA_NOALLOC_MAX_ELEMENTS 128     /* largest m and n */
#define BEM_ACA_NOALLOC_SCRATCH_BYTES 4718592 /* 4.5 MiB of device memory per GPU */
int bem_aca_matrix_noalloc(bem_ctx *ctx, int32_t prec, int32_t m, int32_t n, const void *A, double tol,
                           int32_t max_cols, int32_t *kc_kk, void *U, void *V);

/* Statistics of a compressed or dense operator. */
int bem_op_stats(const bem_op *op, bem_stats *st);

/* All-frequency product (the face-fibre form of eq. (3DacaMult) per frequency):
 * y[r][l] = A(s_l) x[r][l] for r < nrhs and every l, where A is the dense or compressed
 * operator.  x, y: [nrhs][L][3K] complex128 (complex64 is not accepted: the product
 * accumulates near field in complex128 and converts far-field partial sums).  With
 * BEM_SHARED_X, x is [nrhs][3K] and used for every l.  With BEM_TRANSPOSE, y = A(s_l)^T x
 * (the fibre of each face applied on the output side; not with BEM_SHARED_X).  x and y must
 * not overlap. */
int bem_apply(bem_op *op, int32_t nrhs, const void *x, void *y, int32_t flags);

/* gCQ weighted sum (eq. (gCQ) / eq. (3DacaMult)): y = sum_l A(s_l) W[l], computed as
 * sum_k H_k (sum_l f_k[l] W[l]) on a compressed operator (plain sum on a dense one).
 * W: [L][3K] complex128, y: [3K] complex128. */
int bem_apply_weighted(bem_op *op, const void *W, void *y, int32_t flags);

/* Options of bem_solve (NULL: tol 1e-8, inner_tol 1e-3, restart 30, max_iter 500,
 * max_refine 10). */
typedef struct bem_solve_opts {
    double tol;          /* target: ||b_l - A(s_l) x_l|| <= tol ||b_l|| for every frequency and
                            right-hand side, residual taken with the fine operator A */
    double inner_tol;    /* relative residual reached by each inner GMRES run on A_inner */
    int32_t restart;     /* Krylov vectors per GMRES cycle (>= 1) */
    int32_t max_iter;    /* inner-operator products in total (>= 1) */
    int32_t max_refine;  /* refinement sweeps after the first (>= 0) */
    int32_t pad;
} bem_solve_opts;

/* Results of bem_solve. */
typedef struct bem_solve_stats {
    int32_t iterations;   /* inner-operator products (each covers all frequencies and
                             right-hand sides) */
    int32_t refinements;  /* fine-operator products (residuals) */
    int32_t converged;    /* 1 when tol was met */
    int32_t pad;
    double rel_residual;  /* max over frequencies and right-hand sides of ||b - A x|| / ||b|| */
    double seconds;       /* wall time of the call */
} bem_solve_stats;

/* Solution of the discrete boundary integral equations at every contour point: the
 * collocation system of Sec. 2.3 (eq. (discrVK) in the Laplace domain, Sec. 2.4), e.g.
 * V(s_l) t_l = (I/2 + K(s_l)) g_l for the tractions of a Dirichlet problem, with b_l the
 * right-hand side computed by bem_apply.  Solves A(s_l) x[r][l] = b[r][l] for every r < nrhs
 * and l: GMRES per column (all columns batched in each product) with re-orthogonalised
 * classical Gram-Schmidt in FP64, inside iterative refinement: each sweep runs GMRES on
 * A_inner d = r (to inner_tol, or, when A_inner is NULL or A, to what tol requires) and adds
 * d to x, then takes the residual r = b - A x with A.  A cheap inner operator (e.g. the
 * mixed-precision compression) with an accurate fine one (FP64 at a tighter eps) gives the
 * fine operator's accuracy at mostly inner-operator cost.
 *   With BEM_TRANSPOSE in flags the systems are A(s_l)^T x = b (the adjoint solves of a
 *   gradient).
 *   A, A_inner: operators of one device with the same K and L (dense, compressed or
 *   matrix-free; A_inner may be NULL or belong to another context); the work runs on A's
 *   context stream.  b, x: [nrhs][L][3K] complex128, mesh order, host or device per flags; x is
 *   overwritten (zero initial guess).  stats may be NULL.  Returns BEM_OK, BEM_WARN_NOCONV
 *   (x holds the last iterate), or an error (BEM_ERR_ARG for bad sizes or options). */
int bem_solve(bem_op *A, bem_op *A_inner, int32_t nrhs, const void *b, void *x, int32_t flags,
              const bem_solve_opts *opts, bem_solve_stats *stats);

/* ---- Matrix-free products and the adjoint of the single layer ------------------------------
 * The dense discrete operators of eq. (discrVK) at the contour points (Sec. 2.3, 2.4) applied
 * without storing them: every entry is recomputed (regular, near and self rules as in
 * bem_entries, FP64).  For meshes whose dense array does not fit, and as the forward and
 * transposed products of a differentiable single layer. */

/* y[r][l] = A(s_l) x[r][l], or A(s_l)^T x[r][l] (plain transpose, no conjugation) when
 * transpose != 0, for op V, K or HK; x, y: [nrhs][L][3K] complex128 in mesh order, host or
 * device per flags (BEM_DEVICE_PTR).  Cost: K^2 L entries per pass of 4 right-hand sides. */
int bem_apply_mf(bem_ctx *ctx, int32_t op, int32_t transpose, int32_t nrhs, const void *x, void *y, int32_t flags);

/* The double layer against continuous piecewise-linear shape functions (Sec. 2.3, eqs.
 * (subspace), (basis): the Dirichlet data of eq. (discreteCollo) are nodal values, and K of
 * eq. (discrVK) integrates T against the hat function phi_n of each node) collocated at the
 * element centroids, entries recomputed (matrix-free, FP64 rules of bem_entries):
 *   y[r][l][3 i + a] = sum_n (K(s_l)[i, n] g[r][l][3 n ..])_a,
 *   K(s_l)[i, n] = sum over the elements j of node n of int_{gamma_j} T(x_i, y) lambda_v(y) dy
 *   (v = position of n in element j, lambda_v its barycentric coordinate).
 * With BEM_FREE_TERM, y also gets C g with C phi_n(x_i) = I/2 * 1/3 for the three nodes of
 * element i.  g: [nrhs][L][3 n_nodes] complex128 (mesh node order), y: [nrhs][L][3K],
 * host or device per flags (BEM_DEVICE_PTR).  Cost: K^2 L (three weights per evaluation). */
int bem_apply_linear_dl(bem_ctx *ctx, int32_t nrhs, const void *g, void *y, int32_t flags);

/* Matrix-free operator (op V, K or HK of eq. (discrVK) in FP64, nothing stored): bem_apply
 * (plain or BEM_TRANSPOSE, not BEM_SHARED_X) recomputes every entry as bem_apply_mf does, with
 * the mesh, material, contour points and quadrature the context holds at the call.  It can be
 * the fine operator of bem_solve, whose residuals are then exact to quadrature while a
 * compressed inner operator (possibly of another context on the same device, e.g. the
 * unperturbed mesh of a finite-difference study) carries the GMRES iterations.
 * bem_apply_weighted, bem_cq_dirichlet, bem_op_dense_copy and batches refuse it (BEM_ERR_ARG);
 * its statistics report 0 bytes.  Errors: BEM_ERR_ARG for another op, BEM_ERR_STATE without
 * mesh, material and contour points or with several components. */
int bem_matrix_free(bem_ctx *ctx, int32_t op, bem_op **out);

/* Adjoint of the single layer (an extension; the paper has no adjoint): the value
 * S = sum_{r, l} w[r][l]^T V(s_l) x[r][l] (no conjugation) and the gradient of Re S with
 * respect to the node coordinates and the material, for the discrete operator of eq.
 * (discrVK) with the context's quadrature (regular, near and self rules), the class of every
 * pair held fixed.  Regular and near pairs are differentiated exactly (chain rule through the
 * Gauss points, also those of the near rule's sub-triangles, the collocation points and the
 * element areas; speeds through the kernel); self pairs by the derivative of the self integral
 * (the gradient of U weighted by lambda_a - 1/3, the speed derivatives of U and the area
 * term, integrated by the polar rule).  Entries are recomputed, never stored.  w, x:
 * [nrhs][L][3K] complex128, mesh order, host or device per flags.  value: [2] (Re, Im S);
 * grad_nodes: [n_nodes][3]; grad_mat: [3] = d/d rho, d/d c_p, d/d c_s; each output may be
 * NULL.  Cost: K^2 L nrhs kernel evaluations with derivatives.  Errors: BEM_ERR_ARG for
 * nrhs < 1, missing buffers or unknown flags; BEM_ERR_STATE without mesh, material and
 * contour points or with several components. */
int bem_adjoint_v(bem_ctx *ctx, int32_t nrhs, const void *w, const void *x, int32_t flags, double *value,
                  double *grad_nodes, double *grad_mat);

/* Adjoint of the double layer (an extension, as bem_adjoint_v): S = sum_{r, l} w[r][l]^T
 * A(s_l) x[r][l] with A = K (op BEM_OP_K) or I/2 + K (BEM_OP_HK, the free term of eq. (SBIE)
 * at the centroids, whose derivative is zero), the traction kernel of Sec. 2.1 against the
 * piecewise-constant basis, and the gradient of Re S with respect to the node coordinates and
 * the material, pair classes held fixed.  Regular and near pairs: chain rule through the Gauss
 * points, the element normal n_j (dn = (I - n n^T)(dP_a x (P_{a+1} - P_{a+2})) / |N|), the
 * area and the collocation point, with the closed-form R- and speed derivatives of the
 * traction kernel (second R-derivatives of A and B included).  Self pairs: the derivative of
 * the principal-value integral (the traction's r-gradient weighted by lambda_a - 1/3, its
 * normal derivative, its speed derivatives and the area term, by the polar rule with the
 * leading parts of the static kernel).  T does not depend on rho: grad_mat[0] = 0.
 * Arguments, layouts and errors as bem_adjoint_v; BEM_ERR_ARG also for another op. */
int bem_adjoint_k(bem_ctx *ctx, int32_t op, int32_t nrhs, const void *w, const void *x, int32_t flags,
                  double *value, double *grad_nodes, double *grad_mat);

/* ---- Batched products of several compressed operators ------------------------------------
 * The all-frequency product of bem_apply (the face-fibre form of eq. (3DacaMult) at every
 * contour point) for up to 16 compressed operators at once, e.g. several meshes sharing one
 * set of L contour points: one merged plan of all their blocks, faces and row chunks, so that
 * each kernel of the product runs once over every operator, frequency and right-hand side
 * (far-face products, row products, row sums, two batched permutations). */
typedef struct bem_batch bem_batch;

#define BEM_BATCH_GRAPH 1  /* bem_batch_create: record the launches of a call in a HIP graph and
                              replay it while the same device buffers and stream come back */
#define BEM_BATCH_TUNE 2   /* bem_batch_create: time the candidate schedules (segment counts,
                              far faces by decreasing rank) and keep the fastest */

/* Schedule and counters of a batch. */
typedef struct bem_batch_info {
    int32_t nops, nrhs, L, K_total;   /* operators, right-hand sides, frequencies, elements */
    int32_t n_groups, n_segments;     /* row chunks of all operators, row-kernel segments */
    int32_t n_far_faces, seg_target;  /* factored faces, segment target of the schedule */
    int32_t persistent, persistent_wgs; /* always 0: every product kernel takes one work item
                                           (segment or face, column tile) per workgroup */
    int32_t far_sorted, graph;        /* far faces by decreasing rank; HIP graph replay on */
    int32_t graph_builds, graph_launches;
    int32_t n_tuned, pad;             /* timed candidates (at most 8) */
    double tune_ms[8];                /* product time of each timed candidate (events, ms, on
                                         at most 512 columns) */
    int32_t tune_segments[8];         /* its segment count */
    double workspace_bytes;           /* device workspace held by the batch */
    double flop;                      /* algorithmic flops of one batched product: 8 per complex
                                         multiply-add of the stored faces and factors with the
                                         columns, and of the fibres with the inputs */
} bem_batch_info;

/* Creates a batch over ops[0 .. nops) (1 <= nops <= 16): compressed operators with the same
 * L on the same device, possibly of different contexts and meshes; nrhs right-hand sides per
 * operator.  The batch holds its plan and a workspace sized for nrhs (no allocation in
 * bem_batch_apply); the operators must stay alive while it does (bem_op_destroy returns
 * BEM_ERR_STATE until the batch is destroyed).  Runs on the stream of ops[0]'s context.
 * Errors: BEM_ERR_ARG (dense operator, different L or device, nops or nrhs out of range),
 * BEM_ERR_NOMEM. */
int bem_batch_create(bem_op *const *ops, int32_t nops, int32_t nrhs, int32_t flags, bem_batch **out);

/* y[o][r][l] = A_o(s_l) x[o][r][l] for every operator o of the batch: x[o], y[o] are
 * [nrhs][L][3 K_o] complex128 in mesh order, host or device per flags (BEM_DEVICE_PTR; a
 * batch created with BEM_BATCH_GRAPH takes device buffers only).  Results equal those of
 * bem_apply on each operator up to the order of the floating-point sums. */
int bem_batch_apply(bem_batch *b, const void *const *x, void *const *y, int32_t flags);

/* Schedule, tuning times and graph counters of a batch. */
int bem_batch_info_get(const bem_batch *b, bem_batch_info *info);

/* Releases a batch (its plan, workspace and graph). */
int bem_batch_destroy(bem_batch *b);

/* Time stepping of the Dirichlet problem (Sec. 2.4) by convolution quadrature on uniform
 * steps with the BDF2 generating function delta(z) = 3/2 - 2 z + z^2/2: the contour points of
 * the context must be s_l = delta(z_l)/dt, z_l = R exp(2 pi i l / L) (BEM_ERR_FREQ
 * otherwise).  The CQ weights omega_k(A) = R^-k / L sum_l A(s_l) exp(-2 pi i k l / L) are never
 * formed: at step n the history sum_{j<n} omega_{n-j}(V) t_j equals sum_l V(s_l) W_l with
 * W_l = 1/L sum_{j<n} z_l^{-(n-j)} t_j, one weighted sum of eq. (3DacaMult) (the structure of
 * eq. (gCQ)), and W_l follows the recurrence W_l <- z_l^-1 (W_l + t_n / L) (the role of the
 * state update eq. (ODEsol)).  Each step solves omega_0(V) t_n = b_n - history by GMRES, the
 * product of omega_0(V) = 1/L sum_l V(s_l) being a weighted sum with equal weights; the
 * right-hand side is b_n = sum_{j<=n} omega_{n-j}(H) g_j (H = I/2 + K), or g_n when H is NULL.
 *   V, H: dense or compressed operators of one context.  g: [N][3K] samples g(t_n),
 *   t_n = n dt, n < N <= L, mesh order; t: [N][3K] tractions out; host or device per flags.
 *   opts: tol, restart, max_iter, max_refine per step (inner_tol unused); stats: totals over
 *   the steps (rel_residual: the worst step).  Returns BEM_OK or BEM_WARN_NOCONV. */
int bem_cq_dirichlet(bem_op *V, bem_op *H, int32_t N, double dt, double R, const void *g, void *t, int32_t flags,
                     const bem_solve_opts *opts, bem_solve_stats *stats);

/* Per-block description of a compressed operator for tests and reports:
 * rows (int64 x 8 per block): row_begin, row_size, col_begin, col_size (cluster order),
 * is_far, rank, dense_fallback, aca_cols_total.  perm: [K] int32, cluster position ->
 * mesh element.  Either pointer may be NULL.  n_blocks gets the number of blocks. */
int bem_op_blocks(const bem_op *op, int64_t *n_blocks, int64_t *rows, int32_t *perm);

/* Partition only (host; works on a host-only context): fills the same block table as
 * bem_op_blocks for the current mesh with the given eta and leaf; rank columns are 0. */
int bem_partition(bem_ctx *ctx, double eta, int32_t leaf, int64_t *n_blocks, int64_t *rows, int32_t *perm);

/* Frequencies selected by 3D-ACA: hist[l] = number of compressed (non-fallback) blocks
 * whose face list contains slice l (Fig. 6 of the paper plots this). */
int bem_op_freq_hist(const bem_op *op, int64_t *hist);

/* Releases an operator and its device memory. */
int bem_op_destroy(bem_op *op);

/* Library version string. */
const char *bem_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BEM_H */
