/*
 * libgeneo: two-level GenEO-type additive Schwarz preconditioner for
 * lowest-order Nedelec (edge) discretisations of the positive Maxwell
 * problem curl(mu^-1 curl E) + gamma eps E = f, n x E = 0 on Gamma_D,
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: Bootland, Dolean, Nataf, Tournier, "A robust and adaptive
 * GenEO-type domain decomposition preconditioner for H(curl) problems in
 * three-dimensional general topologies" (arXiv 2311.18783).
 *
 * Conventions (every call):
 *   - indices are int32, 0-based; user-visible reals are FP64;
 *   - every call returns 0 (GENEO_OK) or a negative geneo_status; no C++
 *     exception crosses the ABI; geneo_last_error() gives the message of the
 *     last failure on a context;
 *   - host arrays passed in are only read during the call and may be freed
 *     afterwards; handles are owned by the library until geneo_free_*;
 *   - "device" pointers are HIP device memory on the context's device
 *     (e.g. torch float64 cuda tensors' data_ptr()), contiguous, in the free
 *     edge order reported by geneo_system_info; work on them is ordered on
 *     the context's stream;
 *   - a context is not thread-safe.
 */
#ifndef GENEO_H
#define GENEO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GENEO_OK = 0,
  GENEO_EINVAL = -1,       /* bad argument, shape or option */
  GENEO_ENOTSPD = -2,      /* a Cholesky pivot was not positive (message names the matrix and pivot) */
  GENEO_ENOCONV = -3,      /* iteration limit reached; info is still filled */
  GENEO_EOOM = -4,         /* device or host allocation failed */
  GENEO_EHIP = -5,         /* a HIP runtime call failed */
  GENEO_EUNSUPPORTED = -6, /* option not supported */
  GENEO_ESYNC = -7         /* a device-side bounded wait expired (kernel finished, results invalid) */
} geneo_status;

typedef struct geneo_ctx geneo_ctx;
typedef struct geneo_system geneo_system;
typedef struct geneo_decomp geneo_decomp;
typedef struct geneo_precond geneo_precond;

/* Tetrahedral mesh (Section 1: Omega with boundary Gamma; Section 4, Numerical results:
 * Cartesian meshes).  Cells group tets (e.g. the 6 tets of a hex); the
 * overlap of the decomposition is grown by whole cells. */
typedef struct {
  int64_t n_nodes;
  const double* xyz;             /* [n_nodes*3] host, node coordinates */
  int64_t n_tets;
  const int32_t* tets;           /* [n_tets*4] host, node ids */
  const int32_t* cell_of_tet;    /* [n_tets] host, cell id per tet, or NULL = one cell per tet */
  int64_t n_bfaces;
  const int32_t* bfaces;         /* [n_bfaces*3] host, boundary triangles */
  const int8_t* bface_dirichlet; /* [n_bfaces] host, 1 = n x E = 0 imposed, 0 = natural condition */
} geneo_mesh;

typedef struct {
  int64_t n;            /* free edges = unknowns (Dirichlet edges eliminated) */
  int64_t nnz;          /* nonzeros of A */
  int64_t n_edges;      /* all edges */
  int64_t n_free_nodes; /* columns of the gradient matrix G */
  int64_t n_cells;
  double assemble_ms;   /* device time of the element + scatter kernels */
} geneo_system_info;

/* --- context --------------------------------------------------------- */

/* Create a context on HIP device `device`.  `hip_stream` is the hipStream_t
 * all work is ordered on; NULL means the device's default (null) stream. */
int geneo_create(geneo_ctx** ctx, int device, void* hip_stream);
void geneo_destroy(geneo_ctx* ctx);
/* NULL ctx: the message of the last failed geneo_create on this thread. */
const char* geneo_last_error(const geneo_ctx* ctx);

/* --- assemble: A = K + gamma M over free edges, and G ------------------ */

/* Assemble the lowest-order Nedelec system of the weak form
 * a(u,v) = int mu^-1 curl u . curl v + gamma eps u . v (Section 2, the
 * bilinear form; Section 1, A U = (K + gamma M) U = f).  mu, eps: host
 * [n_tets], piecewise constant, > 0; gamma > 0.  Edges are oriented from the
 * lower to the higher node id and numbered lexicographically; edges and
 * nodes of Dirichlet triangles are eliminated.  G (free edges x free nodes)
 * holds -1 / +1 at an edge's first / second node: the gradient matrix whose
 * range is the kernel of the discrete curl-curl part (Section 1). */
int geneo_assemble(geneo_ctx* ctx, const geneo_mesh* mesh, const double* mu,
                   const double* eps, double gamma, geneo_system** out);
int geneo_system_info_get(const geneo_system* sys, geneo_system_info* info);
/* Copy A to host CSR arrays (rowptr [n+1], colind [nnz], vals [nnz]) and the
 * global edge id of each free edge (free_edge_ids [n]).  Any pointer may be NULL. */
int geneo_system_export(geneo_ctx* ctx, const geneo_system* sys, int32_t* rowptr,
                        int32_t* colind, double* vals, int32_t* free_edge_ids);
/* y = A x, device vectors of length n. */
int geneo_spmv(geneo_ctx* ctx, const geneo_system* sys, const double* x, double* y);

/* --- partition: overlapping subdomains, restriction, partition of unity -- */

typedef enum { GENEO_PART_BOX = 0, GENEO_PART_RCB = 1, GENEO_PART_EXPLICIT = 2 } geneo_part_kind;

typedef struct {
  int32_t kind;              /* geneo_part_kind */
  int32_t box[3];            /* BOX: px, py, pz boxes over the bounding box, by cell centroid */
  int32_t nparts;            /* RCB: number of parts */
  const double* rcb_jitter;  /* RCB: [nparts-1] host, relative shift of each split, preorder */
  const int32_t* part_of_cell; /* EXPLICIT: [n_cells] host */
  int32_t overlap;           /* layers of vertex-adjacent cells added (Section 4, Numerical results: one layer) */
} geneo_partition_opts;

typedef struct {
  int32_t n_sub;
  int32_t n_min, n_max;      /* smallest / largest n_i */
  int64_t sum_n;             /* sum of n_i */
  int64_t sum_p;             /* sum of local free-node counts (SNK columns, paper convention) */
  int32_t n_floating;        /* subdomains with a floating component */
  double sum_n3_over_3;      /* sum n_i^3 / 3: Cholesky flops of the local factors */
} geneo_decomp_info;

/* Build the overlapping decomposition (Section 2: Omega_i, N_i, R_i, the
 * partition of unity sum R_i^T D_i R_i = I).  Each non-overlapping part
 * grows by `overlap` layers of cells sharing a vertex.  D_i: chi_i / sum_j
 * chi_j with chi_i = 1 on the nodes of the original cells of part i and
 * 1 - d/overlap on nodes first reached by layer d, averaged over the two
 * ends of an edge. */
int geneo_partition(geneo_ctx* ctx, const geneo_system* sys,
                    const geneo_partition_opts* opts, geneo_decomp** out);
int geneo_decomp_info_get(const geneo_decomp* dec, geneo_decomp_info* info);
/* Subdomain i: n_i, and optionally (host) its free-edge list N_i [n_i]
 * (sorted), its PoU D_i [n_i], its G_i column nodes [p_i] (free-node ids;
 * floating components lose their lowest node). */
int geneo_decomp_subdomain(const geneo_decomp* dec, int32_t i, int32_t* n_i, int32_t* dofs,
                           double* pou, int32_t* p_i, int32_t* gnodes);

/* --- setup: local factors, GenEO eigenproblems, coarse space ------------ */

typedef enum { GENEO_FP64 = 0, GENEO_FP32_REFINE1 = 1 } geneo_precision;
/* Coarse space (Section 4, Numerical results, compares these variants): the split near-kernel
 * columns R_i^T D_i G_i with the GenEO vectors (the method), the split near-kernel columns alone
 * (tau = infinity), none (one-level additive Schwarz), the global near-kernel columns G (the
 * gradients of the free nodes) alone or with the GenEO vectors. */
typedef enum { GENEO_COARSE_SNK_GENEO = 0, GENEO_COARSE_SNK = 1, GENEO_COARSE_NONE = 2,
               GENEO_COARSE_NK = 3, GENEO_COARSE_NK_GENEO = 4 } geneo_coarse_kind;
/* One-level term of the preconditioner: sum_i R_i^T A_i^-1 R_i (eq. (AS), symmetric: PCG) or the
 * restricted sum_i R_i^T D_i A_i^-1 R_i with the partition of unity (eq. (RAS), not symmetric:
 * use GMRES). */
typedef enum { GENEO_WEIGHT_IDENTITY = 0, GENEO_WEIGHT_POU = 1 } geneo_one_level_weight;
/* Elimination order of the coarse columns in the factorisation of E (the
 * coarse space and its span do not depend on it; which columns the greedy
 * basis test leaves out may): subdomain groups (SNK columns, then GenEO
 * columns) in nested-dissection order of the subdomain coupling graph, or
 * all SNK columns subdomain by subdomain followed by all GenEO columns.
 * AUTO (default): nested dissection when the dependency chain of the coarse
 * triangular solves it predicts (from the subdomain adjacency) is at most
 * 0.6 of the natural order's block-row count, else natural. */
typedef enum { GENEO_ORDER_NATURAL = 0, GENEO_ORDER_NESTED_DISSECTION = 1, GENEO_ORDER_AUTO = 2 } geneo_coarse_order;
/* Launch schedule of the block-sparse coarse factorisation (same arithmetic
 * per tile; only the grouping of tile updates, and so their rounding order,
 * differs): STEPS = one block column after another (panel groups of
 * trailing updates); LEVELS = the block columns of equal height in the
 * factor's elimination tree together (one launch for their diagonal blocks,
 * one for their column tiles), levels taken in groups of eight whose
 * updates of later columns are applied once per group (on a chain, one
 * column per level, this is STEPS with groups of eight).  AUTO (default):
 * LEVELS. */
typedef enum { GENEO_SCHEDULE_AUTO = 0, GENEO_SCHEDULE_STEPS = 1, GENEO_SCHEDULE_LEVELS = 2 } geneo_coarse_schedule;

typedef struct {
  double tau;               /* GenEO threshold, keep lambda > tau (Section 4, Numerical results: 10) */
  int32_t nev_max;          /* at most this many eigenvectors per subdomain */
  int32_t coarse;           /* geneo_coarse_kind */
  int32_t local_precision;  /* geneo_precision of the local factors and solves */
  double lobpcg_tol;        /* ||Atilde x - theta B x|| / (|theta| ||B x||) target (default 1e-8) */
  int32_t lobpcg_maxit;
  int32_t lobpcg_guard;     /* extra block vectors beyond nev_max */
  uint64_t seed;            /* random start blocks */
  double coarse_drop_tol;   /* relative Schur pivot below which a coarse column is dependent (default 1e-7) */
  const double* warm_start; /* host [sum_i n_i * nev_max] start blocks (column-major per subdomain) or NULL */
  double fp32_rho_max;      /* FP32_REFINE1: a subdomain whose estimated rho(I - Ahat_i^-1 A_i) exceeds this
                               is factored in FP64 instead (default 0.5; must be < 1) */
  const struct geneo_model* model; /* learned warm start of the eigensolver, or NULL (cold random start);
                               ignored when warm_start is given */
  int32_t keep_ritz;        /* 1: keep the final Ritz block for geneo_model_collect */
  int32_t coarse_order;     /* geneo_coarse_order (default AUTO) */
  int32_t one_level_weight; /* geneo_one_level_weight (default identity) */
  int32_t classical;        /* 1: GenEO vectors from the classical pencil D_j A_j D_j V = lambda A_j^Neu V
                               (Section 3.2, eq. (eigGenEOClassis): no projection out of span(G_j)), an
                               ablation of the method's filtered pencil; default 0 */
  int32_t coarse_schedule;  /* geneo_coarse_schedule (default AUTO) */
} geneo_setup_opts;

typedef struct {
  int32_t n0;               /* coarse columns (SNK + GenEO) */
  int32_t n0_rank;          /* columns kept as a basis */
  int32_t n0_local_dropped; /* SNK columns left out before assembling E: dependent within their node's group */
  int32_t n_snk;            /* SNK columns */
  int32_t n_geneo;          /* GenEO columns */
  int32_t lobpcg_iters;     /* LOBPCG iterations (max over subdomains) */
  int32_t lobpcg_unconverged; /* subdomains whose selected Ritz pairs were not converged at exit */
  int32_t fp64_fallbacks;   /* FP32 local factors replaced by FP64 (all of them when fewer than 1 in 8 would stay FP32) */
  double min_kept_pivot;    /* smallest relative Schur pivot kept in the coarse factor */
  double max_dropped_pivot; /* largest relative Schur pivot dropped */
  double t_extract_ms, t_factor_ms, t_gevp_ms, t_coarse_build_ms, t_coarse_factor_ms; /* device times */
  double local_factor_flops; /* sum n_i^3/3 */
  double fp32_rho_est;      /* FP32_REFINE1: largest probe estimate of rho(I - Ahat_i^-1 A_i) (infinite when
                               fewer than 1 in 8 FP32 factorisations completed: no probe is run), else 0 */
  double coarse_factor_flops; /* flops of the coarse factorisation (on its block-sparse fill pattern) */
  double coarse_fill;       /* fraction of the lower 128 x 128 tiles of E in that pattern (1 = dense) */
  int32_t learned_starts;   /* subdomains whose eigensolver continued from the model's start block: after
                               one Rayleigh-Ritz step on both the model's block and the random block, the
                               largest eigen-residual of the pairs that decide the coarse space (Ritz values
                               above tau, at most nev_max, of either block, plus the next one) was below half
                               that of the random block (otherwise the random block is kept: the cold start) */
  double start_residual;    /* largest eigen-residual of the top nev_max Ritz pairs after the first
                               Rayleigh-Ritz step (start-block quality) */
  int32_t fp32_prechecked;  /* FP32_REFINE1: subdomains factored in FP64 without an FP32 attempt, because
                               0.2 u32 kappa_lb_i > fp32_rho_max (u32 = 2^-24); counted in fp64_fallbacks */
  double fp32_kappa_lb;     /* FP32_REFINE1: largest kappa_lb_i, the lower bound on the condition number of
                               D^-1/2 A_i D^-1/2 (D = diag A_i) from the Rayleigh quotient of a node's
                               gradient (sampled nodes whose edges all lie in Omega_i; 0 if none) */
  int32_t learned_candidates; /* subdomains for which the model proposed a start block (those that fit its
                               canvas); learned_starts of them were kept */
  int32_t coarse_nd_levels; /* depth of the nested dissection of the subdomain graph (0: natural order) */
  int32_t coarse_nd_predicted_depth; /* AUTO: the solve depth predicted for the nested-dissection order */
  int32_t coarse_solve_depth; /* longest chain of dependent 128-row blocks in a coarse triangular solve */
  int32_t coarse_levels;    /* height + 1 of the coarse factor's block elimination tree */
  int32_t coarse_schedule_used; /* geneo_coarse_schedule the factorisation ran with (STEPS or LEVELS) */
  double t_factor_fp32_ms;  /* FP32_REFINE1: device time of the FP32 factorisation of all local matrices alone
                               (part of t_factor_ms, which also holds the check, the probe and any fallback) */
  double coarse_lambda_min; /* estimate of the smallest eigenvalue of the factored coarse matrix (kept columns)
                               scaled by its diagonal, diag(E)^-1/2 E diag(E)^-1/2 (power iteration on the
                               factor's inverse); below 1e-20 the columns are eliminated again */
  double coarse_drop_tol_used; /* drop tolerance of the final coarse factor: coarse_drop_tol times 10 per
                                  re-elimination */
  int32_t coarse_refactors; /* re-eliminations with a tenfold tolerance (0 .. 4) */
  double t_coarse_refactor_ms; /* device time from the end of the first coarse factorisation to the end of the
                                  last (estimates, refills of E, re-eliminations; 0 without re-elimination) */
  double coarse_solve_bytes; /* algorithmic bytes of one coarse solve: every tile of the factor's pattern read
                                once per sweep (forward and backward), 128 x 128 FP64 each */
  double t_lobpcg_loop_ms;  /* device time of the eigensolver's iteration loop (part of t_gevp_ms, which also
                               holds the Neumann factorisation, the node matrices and the start block) */
  double lobpcg_solve_ms;   /* device time of one application of B^-1 = (A_j^Neu)^-1 to the block of k
                               vectors of every subdomain (forward and backward sweep), on the second
                               iteration (0 if the loop stopped after one) */
  double lobpcg_solve_bytes; /* algorithmic bytes of that application: each local Neumann factor's lower
                                triangle read once per sweep, sum n_j (n_j + 1) 8 */
} geneo_precond_info;

void geneo_setup_opts_default(geneo_setup_opts* o);
/* Build M_AS,2^-1 = Z E^-1 Z^T + (I - P_0) sum_i R_i^T A_i^-1 R_i (I - P_0^T)
 * (Section 2, eq. (AS2); Section 3.2, the explicit form of M_AS,2) with
 * A_i = R_i A R_i^T factored by dense Cholesky, and Z spanning the split
 * near-kernel space span(R_i^T D_i G_i) (Definition "Split near-kernel
 * coarse space") plus, per subdomain, the vectors R_j^T D_j (I - xi_j) V
 * of the generalised eigenproblem
 *   (I - xi_j^T) D_j A_j D_j (I - xi_j) V = lambda A_j^Neu V,  lambda > tau
 * (Section 3.2, GEVP with eq. (eigAtildeBAS)); xi_j is the A_j-orthogonal
 * projection on span(G_j).  E = Z^T A Z is factored in FP64; columns of Z
 * that are dependent on earlier ones (relative Schur pivot <= drop tol) are
 * left out of the basis. */
int geneo_setup(geneo_ctx* ctx, const geneo_system* sys, const geneo_decomp* dec,
                const geneo_setup_opts* opts, geneo_precond** out);
int geneo_precond_info_get(const geneo_precond* pc, geneo_precond_info* info);
/* Eigenvalues (descending) found for subdomain i: writes up to `cap` values,
 * *count = number written, *selected = number entering the coarse space. */
int geneo_precond_eigs(const geneo_precond* pc, int32_t i, double* lam, int32_t cap,
                       int32_t* count, int32_t* selected);

/* Ritz vectors of subdomain i (setup with keep_ritz = 1): V [n_i x k]
 * column-major (host), the top-k of the final eigensolver block in
 * descending Ritz-value order, A_i^Neu-orthonormal (Section 3.2 GEVP);
 * k = min(cap, block width); *k_out = columns written. */
int geneo_precond_ritz(geneo_ctx* ctx, const geneo_precond* pc, int32_t i, double* V, int32_t cap,
                       int32_t* k_out);

/* z = M_AS,2^-1 r, device vectors of length n (the paper's preconditioner). */
int geneo_apply(geneo_ctx* ctx, const geneo_precond* pc, const double* r, double* z);

/* --- solve: preconditioned Krylov iteration ------------------------------ */

typedef enum { GENEO_SOLVER_PCG = 0, GENEO_SOLVER_GMRES = 1 } geneo_solver;
/* How PCG applies the two-level preconditioner.  DEFLATED (default): from
 * x0 = Q b with (I - Q A) M_AS + Q, Q = Z E^-1 Z^T, M_AS = sum_i R_i^T A_i^-1 R_i
 * (one coarse solve per iteration); in exact arithmetic PCG then produces the
 * iterates of PCG with M_AS,2 (eq. (AS2)) from x0 = 0, since every residual has
 * Z^T r = 0, where the two operators agree.  BALANCED: M_AS,2 itself from
 * x0 = 0 (two coarse solves per iteration).  geneo_apply always applies
 * M_AS,2; GMRES always uses M_AS,2. */
typedef enum { GENEO_PCG_DEFLATED = 0, GENEO_PCG_BALANCED = 1 } geneo_pcg_form;

typedef struct {
  double rtol;      /* stop at the first k with ||r_k||_2 <= rtol ||b||_2 */
  int32_t maxit;
  int32_t graph;    /* 1: from the second iteration on, replay one iteration (preconditioner apply,
                       products, updates, copy of ||r||^2 to the host) captured as a HIP graph, on a
                       stream of the library's own that is ordered after the context stream's earlier
                       work and before its later work; 0: launch kernel by kernel on the context
                       stream.  Both run the same kernels in the same order (bitwise equal results). */
  int32_t method;   /* geneo_solver: PCG (default; needs the symmetric preconditioner) or right-preconditioned
                       GMRES (Section 4, Numerical results: the paper's Krylov method), whose residual is the
                       true residual b - A x; graph is ignored for GMRES */
  int32_t restart;  /* GMRES: restart length (0: no restart, up to maxit Arnoldi vectors) */
  int32_t true_residual; /* PCG: 1 = once the recurrence residual meets rtol, continue from the true residual
                            b - A x with a fresh direction while that misses rtol (at most twice; then
                            GENEO_ENOCONV); 0 (default) = stop on the recurrence residual.  The true residual
                            is computed and reported either way.  In FP64 it cannot go below about
                            u ||A|| ||x|| / ||b|| (u = 2^-53), which exceeds 1e-8 when gamma is small. */
  int32_t pcg_form;      /* geneo_pcg_form (default DEFLATED) */
} geneo_solve_opts;

typedef struct {
  int32_t iterations;
  double rel_residual;   /* PCG: the recurrence residual ||r_k|| / ||b|| at exit; GMRES: the rotated
                            right-hand side, which is the true residual in exact arithmetic */
  double solve_ms;       /* device wall time of the iteration */
  int32_t graph_replays; /* iterations run as graph replays */
  int32_t residual_replacements; /* PCG with true_residual: restarts from the true residual after the
                            recurrence residual met rtol but b - A x did not (at most 2) */
  double true_rel_residual; /* PCG: ||b - A x|| / ||b|| computed on the device when the recurrence residual
                            met rtol (0 if it never did) */
  double residual_floor; /* PCG: (m + 1) u || |b| + |A| |x| || / ||b|| (m = longest row of A, u = 2^-53): the
                            bound on the rounding error of that computed true residual; a true residual at
                            or below it is as small as FP64 can certify */
  double coarse_solve_ms; /* PCG: device time of one coarse solve (forward and backward sweeps), the mean of
                             the first two (HIP events) */
  int64_t coarse_solves;  /* PCG: coarse solves run (DEFLATED: one per preconditioner application plus the
                             start x0 = Q b; BALANCED: two per application) */
} geneo_solve_info;

/* Solve A x = b (Section 1, the discrete system) from x0 = 0 with PCG
 * preconditioned by pc (or plain CG if pc is NULL), stopping at the first k
 * with ||r_k||_2 <= rtol ||b||_2 for the recurrence residual (see
 * true_residual for the true one); or, with method = GMRES, with
 * right-preconditioned GMRES (Arnoldi on A M^-1 with classical Gram-Schmidt
 * applied twice, Givens rotations; x = M^-1 V y), the solver of Section 4,
 * Numerical results.  b, x: device, length n.  Returns GENEO_ENOCONV at
 * maxit with info filled and the last iterate in x. */
int geneo_solve(geneo_ctx* ctx, const geneo_system* sys, const geneo_precond* pc,
                const double* b, double* x, const geneo_solve_opts* opts, geneo_solve_info* info);

/* --- learned warm start of the eigensolver ------------------------------ */
/* The paper computes the GenEO eigenvectors from scratch in every subdomain
 * (Section 3.2); the model below predicts start blocks for the eigensolver
 * from the subdomain's coefficients.  A subdomain of a hexahedral mesh
 * (cells split into six tetrahedra along the main diagonal) is placed,
 * centred, on a canvas of C^3 cells; the input is, per canvas cell,
 * log mu, log eps, occupancy, "owned by the subdomain before overlap" and
 * the fraction of its nodes on the Dirichlet boundary, plus log10 gamma and
 * a constant; the output is k values per canvas edge (start vectors over
 * the subdomain's edges).  Network: in -> hidden -> hidden -> rows*k, ReLU,
 * BF16 weights and activations, FP32 accumulation; trained with Adam on the
 * span loss ||Y^T Y||_F^2 - 2 ||V^T Y||_F^2 + k (minimal, 0, when
 * Y Y^T = V V^T) against the top-k eigenvectors V (orthonormalised) found
 * by the eigensolver.  A subdomain that does not fit the canvas keeps the
 * random start. */
typedef struct geneo_model geneo_model;

typedef struct {
  int32_t canvas;   /* C: canvas cells per axis (default 12) */
  int32_t hidden;   /* hidden width (default 256) */
  int32_t k;        /* start vectors per subdomain (default 20) */
  uint64_t seed;    /* weight initialisation */
} geneo_model_opts;

typedef struct {
  int32_t in_dim, rows, k, hidden, canvas;
  int64_t n_params;
  int32_t n_train, n_holdout;   /* collected samples */
} geneo_model_info;

typedef struct {
  int32_t epochs, batch;
  double lr;
  uint64_t seed;    /* sample order */
} geneo_train_opts;

typedef struct {
  double loss_first, loss_last;   /* mean training loss of the first and last epoch */
  double holdout_loss;            /* mean loss on the held-out samples after training (0 if none) */
  double train_ms;
} geneo_train_info;

void geneo_model_opts_default(geneo_model_opts* o);
int geneo_model_create(geneo_ctx* ctx, const geneo_model_opts* opts, geneo_model** out);
int geneo_model_info_get(const geneo_model* m, geneo_model_info* info);
/* Append one sample per subdomain of a finished setup (built with
 * keep_ritz = 1 on a hexahedral mesh): its canvas features and its top-k
 * Ritz vectors.  holdout = 1 keeps them out of training (evaluation only). */
int geneo_model_collect(geneo_ctx* ctx, geneo_model* m, const geneo_system* sys, const geneo_decomp* dec,
                        const geneo_precond* pc, int32_t holdout);
int geneo_model_train(geneo_ctx* ctx, geneo_model* m, const geneo_train_opts* opts, geneo_train_info* info);
/* Kernel-level entries (host arrays, row-major): predictions Y [batch x rows*k]
 * for features X [batch x in_dim]; the loss (mean over the batch) and its
 * gradients [n_params] in the order W1 (hidden x in), b1, W2, b2, W3
 * (rows*k x hidden), b3 for targets V [batch x rows*k] and row masks
 * [batch x rows] (V orthonormal on the masked rows). */
int geneo_model_predict(geneo_ctx* ctx, const geneo_model* m, int32_t batch, const float* X, float* Y);
int geneo_model_loss_grad(geneo_ctx* ctx, const geneo_model* m, int32_t batch, const float* X, const float* V,
                          const uint8_t* mask, double* loss, float* grad);
/* Parameters in the gradient order: get returns the BF16 values in use (as
 * float); set rounds to BF16 and resets the optimiser state. */
int geneo_model_get_params(const geneo_model* m, float* params);
int geneo_model_set_params(geneo_ctx* ctx, geneo_model* m, const float* params);
int geneo_model_save(const geneo_model* m, const char* path);
int geneo_model_load(geneo_ctx* ctx, const char* path, geneo_model** out);
void geneo_free_model(geneo_model* m);

/* --- kernel-level entry: batched dense Cholesky ------------------------ */

/* Factor `batch` symmetric positive definite matrices in place, A_b = L_b L_b^T,
 * the dense local factorisation of the method.  A: device, matrix b is
 * column-major n_b x n_b with leading dimension ld_b = n_b rounded up to 128,
 * starting at element offset off_b (off_b multiple of 32); only the lower
 * triangle is read and written; pad rows/columns must hold the identity.
 * precision: GENEO_FP64 (A is double*) or GENEO_FP32_REFINE1 (A is float*).
 * On a non-positive pivot returns GENEO_ENOTSPD naming the matrix and pivot. */
int geneo_potrf_batched(geneo_ctx* ctx, int32_t batch, const int32_t* n_host,
                        const int64_t* off_host, void* A, int32_t precision, double* elapsed_ms);

/* --- autotuner of the batched factorisation schedule -------------------- */

/* Schedule of a batched Cholesky: mode = tile mode of the trailing updates
 * (0: 64 x 64 tile per wave, 4 waves, operands from L2; 1: 8 waves; 2:
 * operands staged through LDS), group = panels per trailing update,
 * potrf = diagonal-block kernel (1: recursive, in FP64 in LDS for both
 * precisions; 0: register kernel in the factor's precision). */
typedef struct {
  int32_t mode, group, potrf;
  double ms;        /* tuner: fastest factorisation time of the batch (ms) */
} geneo_factor_schedule;

/* Time every candidate schedule (tile modes 0-2, groups 4/8/16, both
 * diagonal-block kernels) on synthetic SPD matrices of the given sizes
 * (device memory of the batch is allocated for the run), keep the fastest
 * (minimum over `reps` runs each) and record it in the process-wide table
 * under (precision, largest block count, floor(log2(batch))): every
 * factorisation planned afterwards (geneo_setup's local and Neumann
 * factors, geneo_potrf_batched) uses the table's schedule for its key, or
 * the nearest tuned block count of its precision and class, else the
 * defaults (0, 8, 1).  *tried = candidates timed. */
int geneo_tune_factor(geneo_ctx* ctx, int32_t batch, const int32_t* n_host, int32_t precision, int32_t reps,
                      geneo_factor_schedule* best, int32_t* tried);
/* The schedule a batch of these sizes gets now (table lookup, no timing). */
int geneo_tune_lookup(int32_t batch, const int32_t* n_host, int32_t precision, geneo_factor_schedule* out);
/* Write the table to / merge it from a text file (one entry per line:
 * precision max_blk class mode group potrf ms; '#' starts a comment). */
int geneo_tune_save(const char* path);
int geneo_tune_load(const char* path);

/* Allocation-free geneo_potrf_batched, for callers that cannot allocate
 * device memory (code under stream capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, layout, results (bitwise) and errors as
 * geneo_potrf_batched; the factorisation plan and the diagonal-block inverses
 * live in a 64 MiB device array per device (held until the process ends)
 * instead of buffers allocated per call.  Limit: the inverses take
 * 2 * 128 * ld_b elements of the factor's type per matrix plus a few hundred
 * bytes of plan per block column, so sum_b ld_b <= ~32,000 in FP64
 * (~64,000 in FP32); a larger batch returns GENEO_EINVAL before any device
 * work.  Calls that overlap on one device share the array and race. */
int geneo_potrf_batched_noalloc(geneo_ctx* ctx, int32_t batch, const int32_t* n_host,
                                const int64_t* off_host, void* A, int32_t precision, double* elapsed_ms);

/* --- lifetime ----------------------------------------------------------- */
void geneo_free_system(geneo_system* sys);
void geneo_free_decomp(geneo_decomp* dec);
void geneo_free_precond(geneo_precond* pc);

#ifdef __cplusplus
}
#endif
#endif /* GENEO_H */
