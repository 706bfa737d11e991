/*
 * hcurl_amg.h -- C ABI of the MI355X (gfx950) structure-preserving H(curl)
 * algebraic multigrid library.
 *
 * Method: Tuminaro & Glusa, "A structure preserving H-curl algebraic multigrid
 * method for the eddy current equations".  For the edge-element system
 * A^(e) u = f (Sec. 1, eq. "discrete eddy") the setup builds, on every level,
 *   - the nodal operator A^(n) = D_h^T A^(e) D_h and a smoothed-aggregation
 *     nodal prolongator P^(n) from caller-given aggregates (Sec. 2, Sec. 3),
 *     or on level 0 a caller-given P^(n) whose aggregates come from Alg. 1,
 *   - the coarse gradient D_H by the Reitzinger-Schoeberl rule on the
 *     piecewise-constant prolongator (Sec. 2 and Sec. 4.1, eq. "revised RS DH"),
 *   - the pattern of P^(e) and its local constraint systems (Alg. 2),
 *   - P^(e) by constrained energy minimisation, projected CG (Sec. 3, Sec. 4,
 *     eq. "min2_hcurl"), which keeps P^(e) D_H = D_h P^(n) (eq. "commute"),
 *   - the Galerkin operator A_H = P^(e)T A^(e) P^(e) (Sec. 2),
 * and the solve runs CG preconditioned by one V-cycle with symmetric Hiptmair
 * smoothing and a direct coarsest solve (Sec. 6.1).
 *
 * Conventions for every call
 *   - Return value: 0 on success, a negative HCURL_E* code otherwise; the
 *     message of the last failure on the calling thread is returned by
 *     hcurl_last_error().  No C++ exception crosses this interface.
 *   - Index types: int64 row pointers, int32 column indices, double values.
 *     Internally nnz of every matrix must stay below 2^31 (HCURL_EINVAL).
 *   - Memory space: opts.mem_space says whether the input arrays of setup and
 *     the f / u vectors of solve are host or device (HIP) pointers.  Inputs are
 *     read during the call and never retained or modified.
 *   - Streams: all work is enqueued on opts.stream (a hipStream_t, NULL = the
 *     null stream); setup and solve return after their work has completed.
 *   - Ownership: a handle owns all the device memory it allocates; release it
 *     with hcurl_amg_destroy.  A handle must not be used by two threads at once.
 */
#ifndef HCURL_AMG_H
#define HCURL_AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HCURL_OK = 0,
  HCURL_EINVAL = -1,       /* malformed input (shapes, D_h rows, diagonal, sizes) */
  HCURL_EHIP = -2,         /* HIP runtime error */
  HCURL_ENOMEM = -3,       /* device allocation failed */
  HCURL_EREDUCIBLE = -4,   /* a local coarse-edge graph stayed disconnected (Sec. 4.2)
                              after 64 rounds of the edge-adding repair */
  HCURL_ENOTSPD = -5,      /* non-positive curvature in projected CG or a failed
                              Cholesky of a local or coarsest system */
  HCURL_EMAXIT = -6,       /* PCG stopped at maxit above the tolerance */
  HCURL_EUNSUPPORTED = -7, /* a size limit of this implementation was exceeded
                              (see hcurl_last_error for which) */
  HCURL_ESTAGNATE = -8,    /* PCG stagnated above the tolerance: an iteration left
                              every entry of the iterate unchanged (the criterion
                              of Sec. 6.2, two consecutive iterates equal) */
  HCURL_EINFEASIBLE = -9   /* the commuting constraint of a row of P^(e) has no
                              finite solution: its right-hand side r_i = (D_h
                              P^(n))_i on T_i is not finite, or (rows without
                              single-node coarse edges) |sum_k r_ik| exceeds
                              1e-10 max(1, sum_k |r_ik|), i.e. P^(n) does not
                              keep constants (Sec. 4.2) */
};

enum { HCURL_MEM_HOST = 0, HCURL_MEM_DEVICE = 1 };
enum { HCURL_EMIN_CG = 0, HCURL_EMIN_JACOBI = 1 };
enum { HCURL_INIT_ONES = 0, HCURL_INIT_GIVEN = 1, HCURL_INIT_MPNN = 2 };
enum { HCURL_AGG_GIVEN = 0, HCURL_AGG_MIS2 = 1 };

/* CSR matrix.  rowptr has nrows+1 entries; column indices sorted per row.
 * val may be NULL where only the pattern is read. */
typedef struct {
  int64_t nrows, ncols, nnz;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
} hcurl_csr;

typedef struct hcurl_amg_s* hcurl_amg;

typedef struct {
  int max_levels;          /* cap on the number of levels, 0 = aggregates decide */
  int coarse_max_rows;     /* stop coarsening once a level has <= this many edges
                              (0 = never stop early); the coarsest level is solved
                              by a dense factorisation and may have at most 1024 rows */
  int emin_iters;          /* energy-minimisation iterations per level (default 10) */
  int emin_method;         /* HCURL_EMIN_CG (projected CG, default) or
                              HCURL_EMIN_JACOBI (projected Jacobi, Sec. 3 eq. "emin iteration") */
  double emin_omega;       /* Jacobi damping (default 0.5, Sec. 6.1) */
  int init_guess;          /* HCURL_INIT_ONES: ones on the pattern then the local
                              min-norm correction (Sec. 6.1); HCURL_INIT_GIVEN:
                              init_values on the level-0 pattern, then the same
                              correction; HCURL_INIT_MPNN: the plain guess plus
                              the correction predicted by opts.mpnn (needs
                              coords), then the same correction.  Coarser levels
                              always start from ones. */
  const double* init_values; /* nnz(P^(e)_0) values in pattern order (mem_space) */
  int emin_iters_given;    /* level-0 iterations when init_guess is
                              HCURL_INIT_GIVEN or HCURL_INIT_MPNN (default 3) */
  const struct hcurl_mpnn_s* mpnn; /* network for HCURL_INIT_MPNN */
  int vcycle_fp32;         /* FP32 form of the V-cycle inside FP64 PCG: smoothers and
                              transfers read FP32 copies of the operators, vectors
                              are FP64 on level 0 and FP32 below, residuals use the
                              FP64 operator, the coarsest solve is FP64.
                              0: off (default).  1: only if FP32 epsilon (2^-23)
                              times every smoothed level's cancellation_ratio is
                              at most 10, else the V-cycle stays FP64
                              (hcurl_amg_stats_t.vcycle_fp32 tells which).
                              2: unconditionally. */
  const hcurl_csr* nodal_prolongator; /* NULL (default), or a level-0 nodal prolongator
                              P^(n), m_h x m_1 with values, in mem_space, used in
                              place of smoothed aggregation (the method takes
                              "P^(n) or aggregates", Sec. 4.1).  Every row is
                              divided by its sum (summed in column order) so that
                              P^(n) keeps constants; an empty row, a zero or
                              non-finite row sum is HCURL_EINVAL.  If aggregates[0]
                              is NULL the level-0 aggregates (the piecewise-constant
                              P-bar behind D_H) come from Alg. 1 as described
                              below; otherwise aggregates[0] must map onto
                              exactly the m_1 columns.  level_info reports rho and
                              omega as 0 for that level. */
  int alg1_passes;         /* passes of Alg. 1 (default 2, >= 1).  Column j gets the
                              target t_j = ceil(nnz(P_:j) m_h / nnz(P)).  In each pass
                              the columns, in order, take their ceil(t_j / passes)
                              still unassigned rows of largest |p_ij| (ties: smaller
                              row).  Rows left over take the column of their largest
                              |p_ij| (ties: smaller column).  Then, columns in order,
                              a column left without rows takes its row of largest
                              |p_ij| (ties: smaller row) among rows whose column keeps
                              another row; if it has none, HCURL_EINVAL. */
  int pbar_alg1;           /* 0 (default): P-bar behind D_H is the piecewise-constant
                              prolongator of the aggregates.  1: P-bar comes from
                              Alg. 1 applied to the smoothed P^(n) of every level, as
                              in the paper's own runs (Sec. 4.1); P^(n) is unchanged. */
  int aggregation;         /* HCURL_AGG_GIVEN (default): levels with a caller map only.
                              HCURL_AGG_MIS2: a level with no map (aggregates[l] NULL,
                              or l >= n_agg_levels) is aggregated on the graph of its
                              A^(n) (not in the paper, which takes aggregates from an
                              SA package): roots form a distance-2 maximal independent
                              set chosen in Luby rounds with priority (bits 30..63 of
                              splitmix64(i), i); every other node joins the root next
                              to it or, two steps away, the aggregate of its neighbour
                              of largest priority among those next to a root; ids
                              follow the roots' order.  Coarsening then stops at
                              coarse_max_rows, max_levels, or a level the aggregation
                              does not reduce. */
  int power_iters;         /* power iterations for rho(D^-1 A^(n)), default 20 */
  int record_energy;       /* 1: measure 1/2 <P, A P> after every emin iteration */
  int emin_codes;          /* 1 (default): the first masked product A X of an energy
                              minimisation records, per product a_ik x_kj, a 2-byte
                              code (the A entry it comes from and the slot of j in
                              row i's pattern), and the later products of that
                              minimisation read the codes back instead of searching.
                              The codes live while the minimisation runs; a level
                              whose codes would take more than 16 GiB or half the
                              free device memory, or whose allocation for them
                              fails with HCURL_ENOMEM, searches.
                              0: every product searches.  Both give the same
                              P^(e) to rounding (the sums are LDS atomics). */
  int profile;             /* 0: off.  1: time every eagerly launched kernel with HIP
                              events (hcurl_amg_kernel_stats); on a non-null stream the
                              V-cycle levels below the finest replay as one HIP graph,
                              booked as "graph_coarse_levels".  2: as 1 with no graphs.
                              3: as 1 in the setup and on every 16th PCG iteration
                              (0, 16, ...); the other iterations run as with 0, so
                              the solve time carries little event overhead. */
  int mem_space;           /* HCURL_MEM_HOST or HCURL_MEM_DEVICE */
  void* stream;            /* hipStream_t */
  /* Device memory of the handle.  NULL (default, both): hipMallocAsync and
     hipFreeAsync on `stream`.  Otherwise dev_alloc(bytes, stream, alloc_ctx)
     returns device memory for use in stream order on `stream` (NULL makes the
     call fail with HCURL_ENOMEM) and dev_free(ptr, bytes, stream, alloc_ctx)
     gives it back; both are called on the thread that calls the library,
     from hcurl_amg_setup, _solve, _vcycle, _update, _commute_residual, the
     exports and hcurl_amg_destroy, never while a graph is being captured.
     Work enqueued on `stream` may still use a buffer when it is freed: the
     allocator must not hand it to other streams before that work completes
     (a stream-ordered pool on the same stream, such as PyTorch's caching
     allocator, does this).  Both functions must stay valid until
     hcurl_amg_destroy returns.  Set both or neither (HCURL_EINVAL).  Training
     samples (hcurl_amg_mpnn_sample) and networks use the default. */
  void* (*dev_alloc)(size_t bytes, void* stream, void* alloc_ctx);
  void (*dev_free)(void* ptr, size_t bytes, void* stream, void* alloc_ctx);
  void* alloc_ctx;
} hcurl_amg_opts;

/* Fills the defaults listed above. */
void hcurl_amg_default_opts(hcurl_amg_opts* opts);

/*
 * hcurl_amg_setup -- build the hierarchy (Alg. 3 on every level).
 *   A       n_h x n_h edge operator A^(e) = S + M, symmetric positive definite,
 *           positive diagonal (Sec. 1, eq. "discrete eddy").
 *   Dh      n_h x m_h discrete gradient: every row two entries, -1 at the tail
 *           node and +1 at the head node (Sec. 1), or a single +-1: a Dirichlet
 *           edge whose other node was eliminated (Sec. 2).  Every coarse node
 *           that a Dirichlet edge's remaining node is aggregated to gets one
 *           single-node coarse edge (+1 at that node), placed after the two-node
 *           coarse edges in node order; Alg. 2 weighs it by W = 2 and the local
 *           systems that hold one keep every column.  The learned initial guess
 *           does not take Dirichlet edges (HCURL_EUNSUPPORTED).
 *   coords  m_h x 3 node coordinates (row-major) or NULL; kept for the learned
 *           initial guess features, not needed otherwise.
 *   aggregates[l]  for l < n_agg_levels: int32 map from the nodes of level l to
 *           aggregate ids 0..m_{l+1}-1, every id used (the non-overlapping
 *           aggregates of Sec. 2).  Level l+1's nodes are level l's aggregates.
 *           aggregates[0] may be NULL when opts.nodal_prolongator is given
 *           (n_agg_levels still counts level 0); with opts.aggregation =
 *           HCURL_AGG_MIS2 any map may be NULL and n_agg_levels may be 0.
 *   out     receives the handle.
 * Errors: HCURL_EINVAL (shapes, D_h rows, non-positive diagonal, aggregate ids),
 * HCURL_EREDUCIBLE, HCURL_ENOTSPD, HCURL_EUNSUPPORTED, HCURL_EHIP, HCURL_ENOMEM.
 */
int hcurl_amg_setup(const hcurl_csr* A, const hcurl_csr* Dh, const double* coords,
                    const int32_t* const* aggregates, int n_agg_levels,
                    const hcurl_amg_opts* opts, hcurl_amg* out);

/*
 * hcurl_amg_solve -- PCG with one V-cycle per iteration (Sec. 6.1), x0 = 0,
 * stopping when ||r||_2 <= rtol ||f||_2 on the recursive residual.
 *   f, u    n_h vectors in opts.mem_space of the handle; u is overwritten.
 *   iters   receives the iteration count; relres the true relative residual
 *           ||f - A u|| / ||f|| (both may be NULL).
 * Returns HCURL_EMAXIT (with u, iters and relres written) if maxit is reached,
 * HCURL_ESTAGNATE (u, iters, relres written) if an iteration leaves every
 * entry of the iterate unchanged before the tolerance is met (Sec. 6.2: the
 * attainable accuracy is limited by rounding; a larger rtol, such as the
 * paper's kappa(D^-1 A) / 1e16 of Sec. 6.1, is then the remedy).
 */
int hcurl_amg_solve(hcurl_amg h, const double* f, double* u, double rtol, int maxit,
                    int* iters, double* relres);

/*
 * hcurl_amg_solve_noalloc -- hcurl_amg_solve for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and errors as
 * hcurl_amg_solve, computed by the same kernels.
 *   A host-memory handle stages f and u through a file-scope device array of
 *   2 * HCURL_NOALLOC_MAX_ROWS doubles (32 MiB) in place of the two per-call
 *   buffers of hcurl_amg_solve; every GPU the library runs this call on keeps
 *   its own copy of that array until the process ends.  A device-memory
 *   handle needs no staging.  Nothing is allocated: a device allocation
 *   requested inside the call fails it with HCURL_EUNSUPPORTED.
 *   The handle's device must be the current device (HCURL_EINVAL otherwise).
 * Errors: those of hcurl_amg_solve, and HCURL_EUNSUPPORTED for a host-memory
 * handle of more than HCURL_NOALLOC_MAX_ROWS edges.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (f and u are written in full before they are read, so nothing
 * needs clearing).  The call returns after its work has completed, so calls
 * made one after another never overlap; calls that overlap on one GPU (two
 * host threads) race on the array and must be serialised by the caller.
 */
#define HCURL_NOALLOC_MAX_ROWS 2097152
int hcurl_amg_solve_noalloc(hcurl_amg h, const double* f, double* u, double rtol, int maxit,
                            int* iters, double* relres);

/* One V-cycle application z = V(r) (FP64 or FP32 per the handle); r, z in
 * the handle's mem_space. */
int hcurl_amg_vcycle(hcurl_amg h, const double* r, double* z);

void hcurl_amg_destroy(hcurl_amg h);

int hcurl_amg_num_levels(hcurl_amg h);

/* Sizes of level l: rows (edges) n, nodes m, nnz of A_l, A^(n)_l and, for
 * l < levels-1, of P^(e)_l, P^(n)_l, T_l, and the number of coarse edges. */
typedef struct {
  int64_t n_edges, n_nodes, nnz_A, nnz_An;
  int64_t nnz_Pe, nnz_Pn, nnz_T, n_coarse_edges;
  int32_t n_colors_A, n_colors_An;
  double rho, omega;       /* power-iteration estimate and SA damping */
  double cancellation_ratio; /* max over nodes u of (|D|^T|A||D| 1)_u / (D^T A D)_uu:
                              the relative rounding error of A x for a gradient
                              field x, in units of the precision of A (0 on the
                              coarsest level) */
  int64_t irreducible_added; /* coarse edges that make_irreducible (Alg. 2) added to
                              D_{l+1} beyond the RS edges; they are merged into the
                              lexicographic edge order */
} hcurl_level_info;

int hcurl_amg_level_info(hcurl_amg h, int level, hcurl_level_info* info);

/* Structure check of level l < levels-1 (the commuting relation of Sec. 4.2,
 * P^(e)_l D_{l+1} = D_l P^(n)_l), computed on the device over every row:
 * abs_max = max |(P^(e) D_{l+1} - D_l P^(n))_iK| and ref_max = max |(D_l P^(n))_iK|
 * over the pattern T_l (which holds both products' patterns).  The library
 * keeps the relation to rounding, so abs_max / ref_max is a small multiple of
 * the FP64 epsilon; a NaN anywhere makes abs_max NaN.  Host outputs.
 * Errors: HCURL_EINVAL (level, NULL outputs, unusable handle). */
int hcurl_amg_commute_residual(hcurl_amg h, int level, double* abs_max, double* ref_max);

/* Galerkin check of the curl-curl part (Sec. 2: the coarse curl-curl operator
 * annihilates the coarse gradient, S_H D_H = 0, because P^(e) D_H = D_h P^(n)
 * and S_h D_h = 0).  S is the caller's curl-curl matrix S_h of level 0, n_0 x
 * n_0 with values, in the handle's mem_space, read during the call.  On the
 * device S_{l+1} = P^(e)_l^T S_l P^(e)_l is formed level by level and, for
 * every level l < nlev (nlev <= levels), abs_max[l] = max |(S_l D_l)_ij| and
 * ref_max[l] = max |(S_l)_ij| are written (host arrays).  abs_max / ref_max
 * is a small multiple of the FP64 epsilon when S_h D_h = 0 holds to rounding.
 * Errors: HCURL_EINVAL (shape, NULL arguments, nlev out of range). */
int hcurl_amg_curl_residual(hcurl_amg h, const hcurl_csr* S, int nlev, double* abs_max, double* ref_max);

/* Export of level data to caller-allocated HOST arrays sized from level_info.
 * which: */
enum {
  HCURL_EXPORT_A = 0,    /* A_l               n x n     */
  HCURL_EXPORT_AN = 1,   /* A^(n)_l           m x m     */
  HCURL_EXPORT_PN = 2,   /* P^(n)_l           m x m_H   */
  HCURL_EXPORT_PE = 3,   /* P^(e)_l           n x n_H   */
  HCURL_EXPORT_R = 4,    /* D_l P^(n)_l on the pattern T_l, n x m_H */
  HCURL_EXPORT_DH = 5,   /* D_{l+1} as CSR   n_H x m_H (-1 tail, +1 head) */
  HCURL_EXPORT_P0 = 6    /* initial guess actually used (after the min-norm
                            correction) on the P^(e)_l pattern */
};
int hcurl_amg_export_csr(hcurl_amg h, int level, int which, int64_t* rowptr, int32_t* col, double* val);

enum {
  HCURL_VEC_COLORS_A = 0,   /* int32[n] colour of every edge row            */
  HCURL_VEC_COLORS_AN = 1,  /* int32[m] colour of every node row            */
  HCURL_VEC_ENERGY = 2,     /* double[iters+1] energies (record_energy = 1) */
  HCURL_VEC_LOCAL_PAIRS = 3, /* uint16[nnz_Pe] local tail | head << 8 in T_i */
  HCURL_VEC_PCG_HISTORY = 4, /* double[iters+1] recursive relative residuals of the
                                last solve (level must be 0) */
  HCURL_VEC_AGGREGATES = 5,  /* int32[m] map of P-bar (the coarse node of every node
                                that D_H is built from): the caller's aggregates, or
                                Alg. 1's (l < levels-1) */
  HCURL_VEC_LS_HISTOGRAM = 6, /* int64[HCURL_LS_HIST_J * HCURL_LS_HIST_NP]: number of
                                rows of P^(e)_l whose local least-squares problem
                                has |J| = |T_i| coarse nodes and n_p pattern entries
                                at [|J| * HCURL_LS_HIST_NP + n_p] (the sub-problem
                                sizes of Table 4; larger values share the last
                                bin of their axis).  Counted on the device. */
  HCURL_VEC_PCG_ALPHA = 7,   /* double[iters] CG step lengths alpha_k of the last
                                solve (level must be 0) */
  HCURL_VEC_PCG_BETA = 8     /* double[iters-1] CG coefficients beta_k of the last
                                solve (level must be 0) */
};
#define HCURL_LS_HIST_J 32
#define HCURL_LS_HIST_NP 512
int hcurl_amg_export_vec(hcurl_amg h, int level, int which, void* out, int64_t capacity_bytes);

/*
 * hcurl_amg_update -- setup reuse for a sequence of related systems: a new edge
 * matrix with the sparsity pattern of the setup's (a time step, a Newton step).
 * The paper suggests both forms: keeping the transfers across solves while
 * re-projecting the matrix (remarks after Table 4), and starting the energy
 * minimisation from the previous prolongator (Sec. 3).  Every pattern (T, the
 * P^(e) pattern, D_H, local graphs) and every colouring is kept.
 *   A      the new matrix, n_h x n_h with the setup's row pointers and columns
 *          (HCURL_EINVAL otherwise), in opts.mem_space; read during the call.
 *   mode   HCURL_REUSE_TRANSFERS: P^(n)_l, P^(e)_l and D_H are kept; A^(n)_l,
 *          A_{l+1} = P^(e)T A_l P^(e), the diagonals, the FP32 copies and their
 *          guard, and the coarsest inverse are recomputed (energies cleared).
 *          HCURL_REUSE_WARM: as above, and on every level the smoothed-
 *          aggregation P^(n) is rebuilt from the new A^(n) (a caller-given
 *          level-0 P^(n) is kept), R = D P^(n) on T follows it, and P^(e)
 *          starts from its previous values, corrected onto the new constraints,
 *          for `iters` projected-CG (or Jacobi, per opts.emin_method) iterations.
 *   iters  iterations for HCURL_REUSE_WARM; < 0 takes opts.emin_iters.
 * Errors: HCURL_EINVAL (pattern, mode, single-level hierarchy), and those of
 * setup.  After a failure part of the hierarchy may already hold the new
 * operators: the handle then refuses solve, vcycle and update (HCURL_EINVAL)
 * and must be destroyed.
 */
enum { HCURL_REUSE_TRANSFERS = 0, HCURL_REUSE_WARM = 1 };
int hcurl_amg_update(hcurl_amg h, const hcurl_csr* A, int mode, int iters);

/* Whole-hierarchy statistics. */
typedef struct {
  int num_levels;
  double operator_complexity;   /* sum nnz(A_l) / nnz(A_0) (Sec. 6.1) */
  double setup_ms;              /* wall time of the last setup */
  double solve_ms;              /* wall time of the last solve */
  int last_iters;
  double last_relres;
  int vcycle_fp32;              /* 1 if the FP32 form of the V-cycle is in use */
  double update_ms;             /* wall time of the last hcurl_amg_update */
  /* Extreme eigenvalue estimates of the preconditioned operator V A from the
     last solve's CG coefficients (Lanczos matrix T_00 = 1/alpha_0, T_jj =
     1/alpha_j + beta_{j-1}/alpha_{j-1}, T_j,j+1 = sqrt(beta_j)/alpha_j).  They
     lie inside V A's spectrum and approach its ends as iterations grow; their
     ratio estimates kappa(V A).  With the FP32 form's flexible beta this is an
     approximation.  0 before the first solve. */
  double lanczos_lambda_min, lanczos_lambda_max;
  int last_stagnated;           /* 1 if the last solve ended with HCURL_ESTAGNATE */
  int max_local_J, max_local_np; /* largest |T_i| and n_p over all levels */
} hcurl_amg_stats_t;

int hcurl_amg_stats(hcurl_amg h, hcurl_amg_stats_t* s);

/* Per-kernel timings (opts.profile = 1): for kernel k < n, its name, launch
 * count, summed milliseconds (HIP events on the handle's stream) and summed
 * algorithmic bytes moved; for the dense network layers, whose names end in
 * "_flop", the summed floating-point operations instead.  Returns the number
 * of kernels recorded. */
int hcurl_amg_kernel_stats(hcurl_amg h, int max_kernels, char (*names)[48], int64_t* launches,
                           double* ms, double* bytes);
void hcurl_amg_reset_kernel_stats(hcurl_amg h);

/*
 * Learned initial guess for P^(e) (level 0).  A message-passing network on the
 * pattern entries e = (i, j) of P^(e) (fine edge i, coarse edge j): 16 input
 * features per entry, hidden width 64, 3 layers; each layer averages the
 * hidden states over the entry's row and column and applies
 * h <- h + silu([h, mean_row, mean_col] W_l + b_l).  The output head gives a
 * correction delta_e added to the plain initial value; the result is always
 * made feasible by the local min-norm correction, so the commuting relation
 * holds exactly whatever the network predicts.  Dense layers run as BF16
 * matrix-core products with FP32 accumulation; master weights are FP32.
 *
 * Parameters are a flat FP32 array in the order W_in (16x64 row-major), b_in
 * (64), then for l = 0..2: W_l (192x64), b_l (64), then w_out (64), b_out (1).
 */
typedef struct hcurl_mpnn_s* hcurl_mpnn;
typedef struct hcurl_mpnn_sample_s* hcurl_mpnn_sample;

int64_t hcurl_mpnn_num_params(void);
/* params: host array of hcurl_mpnn_num_params() floats, copied. */
int hcurl_mpnn_create(const float* params, void* stream, hcurl_mpnn* out);
int hcurl_mpnn_get_params(hcurl_mpnn net, float* params);
/* Debug form of the dense products (on = 1): FP32 operands and master weights
 * with plain FMAs in place of BF16 matrix-core products (weight gradients
 * summed over the entries in FP64).  Forward, loss and gradients then agree
 * with an FP64 evaluation of the same network to about 1e-5, which checks the
 * structure of the forward and backward kernels apart from BF16 rounding.
 * Slow: one thread per output.  on = 0 restores the BF16 products. */
int hcurl_mpnn_set_fp32_products(hcurl_mpnn net, int on);
void hcurl_mpnn_destroy(hcurl_mpnn net);

/* Training sample from a hierarchy built with HCURL_INIT_ONES and coords:
 * the level-0 features, the pattern graph, the plain initial values and the
 * target = the final P^(e)_0 values.  The sample owns device copies. */
int hcurl_amg_mpnn_sample(hcurl_amg h, hcurl_mpnn_sample* out);
int64_t hcurl_mpnn_sample_entries(hcurl_mpnn_sample s);
/* host copies: features (E x 16 floats), p0 and target (E doubles); any may be NULL */
int hcurl_mpnn_sample_export(hcurl_mpnn_sample s, float* features, double* p0, double* target);
void hcurl_mpnn_sample_destroy(hcurl_mpnn_sample s);

/* delta (E doubles, host) predicted for the sample */
int hcurl_mpnn_forward(hcurl_mpnn net, hcurl_mpnn_sample s, double* delta);
/* loss = mean_e (p0_e + delta_e - target_e)^2 and its gradient (host,
 * hcurl_mpnn_num_params() floats; grad may be NULL) */
int hcurl_mpnn_loss_grad(hcurl_mpnn net, hcurl_mpnn_sample s, double* loss, float* grad);
/* one Adam step (step counts from 1) on the sample; returns the loss before it */
int hcurl_mpnn_train_step(hcurl_mpnn net, hcurl_mpnn_sample s, float lr, float beta1, float beta2, float eps, int step,
                          double* loss);

const char* hcurl_last_error(void);
const char* hcurl_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif
