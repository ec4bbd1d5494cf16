/*
 * qmg -- shifted solves (Q - tau I) x = b for the Hermitian Wilson(-clover)
 * Dirac operator Q = Gamma5 D on one MI355X (gfx950).
 *
 * The operation is the inner solve of the GD-lambda-AMG eigensolver of
 * Frommer, Kahl, Knechtli, Rottmann, Strebel, Zwaan (arXiv:2004.08146):
 * the correction equation (eq. (1.1) / eq. (3.3)), solved in its
 * Gamma5-preconditioned form (D - tau Gamma5) x = Gamma5 b (eq. (3.6) <=> eq. (3.7)) by
 * FGMRES with a two-level aggregation multigrid preconditioner (Sec. 2)
 * whose smoother is red-black SAP (Sec. 2, eq. (2.10)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice dims[4] = {N0 (time), N1, N2, N3}; canonical site index
 * ((x0*N1 + x1)*N2 + x2)*N3 + x3; periodic in all directions.
 * Canonical spinor: complex128 [V][4 spin][3 colour] (interleaved re, im).
 * Canonical gauge field: complex128 [V][4 mu][3][3]; U[x][mu] multiplies
 * psi(x + mu) in the forward hop of eq. (2.5).
 * Gamma basis: chiral, gamma5 = diag(1, 1, -1, -1) (Sec. 2);
 * gamma0 = [[0,-I],[-I,0]], gamma_k = [[0,-i sigma_k],[i sigma_k,0]].
 *
 * Internal ("packed") fields live on the device in a block-major layout
 * private to the library: produce them with qmg_pack, read them back with
 * qmg_unpack; qmg_field_bytes gives the size of one field.  nrhs fields are
 * stored back to back.  Precisions: QMG_F64 (double), QMG_F32 (float),
 * QMG_BF16 (bfloat16 storage, float arithmetic).
 * Coarse vectors (restrict / prolong / apply_coarse) are complex
 * [nrhs][nblocks][2*ntv] in double for QMG_F64 and float otherwise, coarse
 * site order as reported by qmg_coarse_site_order.
 *
 * Ownership: every pointer argument is owned by the caller; unless stated
 * otherwise pointers to fields are DEVICE pointers on the context's device
 * and tau arrays are HOST pointers.  The library copies what it keeps
 * (gauge field, clover term, interpolation, coarse operator) and holds no
 * caller pointer after a call returns.  Workspace is allocated lazily and
 * released by qmg_destroy.
 *
 * Asynchrony: compute calls enqueue on `stream` and return without waiting,
 * except qmg_set_gauge, qmg_set_test_vectors, qmg_setup_mg, qmg_field_dot,
 * qmg_coarse_solve, qmg_vcycle, qmg_solve_shifted and qmg_autotune, which
 * synchronise the stream.
 *
 * Errors: the return code is the only channel (no C++ exception crosses the
 * interface); qmg_last_error gives a message.  A context is not thread safe.
 */
#ifndef QMG_H
#define QMG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qmg_ctx qmg_ctx;

typedef enum {
  QMG_OK = 0,
  QMG_NOT_CONVERGED = 1, /* warning: outputs are valid, tolerance not reached */
  QMG_E_ARG = -1,        /* invalid argument (sizes, pointers, blocking) */
  QMG_E_STATE = -2,      /* call needs state not set yet (gauge, multigrid) */
  QMG_E_NOMEM = -3,      /* device allocation failed */
  QMG_E_HIP = -4,        /* HIP runtime error */
  QMG_E_NUMERIC = -5     /* NaN/Inf or breakdown detected */
} qmg_status;

typedef enum { QMG_F64 = 0, QMG_F32 = 1, QMG_BF16 = 2 } qmg_prec;

/* Solver parameters (defaults from the paper's parameter table and readings:
 * qmg_default_params). */
typedef struct {
  double tol;          /* stop at ||b - (Q - tau) x|| / ||b|| <= tol (1e-10) */
  int maxiter;         /* max FGMRES iterations (preconditioner applications) */
  int restart;         /* FGMRES restart length m */
  int nu_post;         /* SAP sweeps after the coarse correction (3) */
  int n_mr;            /* minimal-residual steps per SAP block solve (3) */
  int coarse_maxiter;  /* max coarse GMRES iterations per V-cycle */
  double coarse_tol;   /* coarse residual reduction (0.5); <= 0: run coarse_maxiter */
  qmg_prec mg_prec;    /* precision of the V-cycle (SAP, transfer, coarse) */
  int use_coarse;      /* 1: two-level V-cycle; 0: SAP only (no coarse level) */
  int use_graph;       /* 1: replay the V-cycle as a captured HIP graph */
  int q_form;          /* 0: the Gamma5-preconditioned form (D - tau Gamma5) x = Gamma5 b, every
                          level built on D - tau Gamma5 (eq. (3.7), the default); 1: FGMRES,
                          SAP and the coarse grid on Q - tau itself (the comparison of Sec. 3.3) */
  int smoother;        /* 0: red-black SAP (nu_post sweeps); 1: GMRES smoothing, nu_post fixed
                          GMRES steps on the fine residual equation (Sec. 2's alternative) */
  int levels;          /* 2 (default), or 3: the coarse correction becomes coarse_maxiter steps of
                          FGMRES on A_c (a K-cycle; a handful, e.g. 4), right-preconditioned by the
                          level-2 cycle (needs qmg_set_level3_vectors / qmg_setup_level3; always
                          fixed steps) */
  int l3_iters;        /* levels = 3: GMRES steps on the level-3 operator per level-2 cycle (8) */
  int l2_smooth;       /* levels = 3: GMRES smoothing steps on level 2 per level-2 cycle (2) */
  int x0;              /* 0 (default): the solve starts from x = 0; 1: the x passed in is the
                          initial guess (FP64 finite values; a solve that stopped at maxiter resumes
                          from its own result, since each restart cycle starts from the true
                          residual of the current x) */
} qmg_params;

#define QMG_STATS_HIST 32  /* entries of qmg_stats.relres_hist */

typedef struct {
  int iters;           /* FGMRES iterations for this right-hand side */
  int restarts;        /* restart cycles */
  int coarse_iters;    /* total coarse GMRES iterations */
  double true_relres;  /* final ||b - (Q - tau) x|| / ||b||, FP64 */
  double seconds;      /* wall time of the whole batched solve */
  /* time of the batched solve by phase, measured with HIP events on the solve's
     stream (the same for every right-hand side of the batch): preconditioner
     (V-cycles), FP64 operator products of the Arnoldi steps, Gram-Schmidt (dot
     products, updates and their host round trips); initial residual, least
     squares and restarts make up the rest of `seconds` */
  double vcycle_seconds;
  double apply_seconds;
  double orth_seconds;
  int n_hist;          /* entries used in relres_hist */
  double relres_hist[QMG_STATS_HIST];  /* true relative residual in FP64 at the start of every
                                          restart cycle this right-hand side took part in, the last
                                          entry being the final one (first QMG_STATS_HIST kept) */
} qmg_stats;

qmg_params qmg_default_params(void);

/* Create a context for lattice dims with Schwarz/aggregation blocks `block`
 * (each extent a power of two dividing the lattice; at most 1024 sites per
 * block) on HIP device `device`.  SAP and multigrid additionally need 16..256
 * sites per block and an even number (>= 2) of blocks per direction
 * (red-black colouring of the blocks, Sec. 2, text after eq. (2.10));
 * apply-only contexts may use a single block per direction.
 * Returns QMG_E_ARG for invalid shapes, QMG_E_HIP if the device is unusable. */
qmg_status qmg_create(qmg_ctx** ctx, const int dims[4], const int block[4], int device);
qmg_status qmg_destroy(qmg_ctx* ctx);
const char* qmg_last_error(const qmg_ctx* ctx);

/* Bytes of one internal spinor field / one coarse vector in precision p. */
size_t qmg_field_bytes(const qmg_ctx* ctx, qmg_prec p);
size_t qmg_coarse_bytes(const qmg_ctx* ctx, qmg_prec p);
/* Lexicographic block index (((X0*NB1+X1)*NB2+X2)*NB3+X3) of every coarse
 * site in library order; out is a HOST array of nblocks entries. */
qmg_status qmg_coarse_site_order(const qmg_ctx* ctx, int64_t* out, int64_t n);

/* Canonical complex128 spinors (device) <-> internal fields of precision p
 * (RNE conversion when narrowing). */
qmg_status qmg_pack(qmg_ctx* ctx, void* dev_internal, const double* canon, int nrhs,
                    qmg_prec p, hipStream_t stream);
qmg_status qmg_unpack(qmg_ctx* ctx, double* canon, const void* dev_internal, int nrhs,
                      qmg_prec p, hipStream_t stream);

/* result[2k], result[2k+1] = Re, Im of <a_k, b_k> = sum conj(a_k) b_k over one
 * field (fixed summation order, accumulated in double); result is a HOST
 * array of 2*nrhs doubles; synchronises the stream. */
qmg_status qmg_field_dot(qmg_ctx* ctx, double* result, const void* a, const void* b, int nrhs, qmg_prec p,
                         hipStream_t stream);

/* As qmg_field_dot, for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): no device
 * allocation of any kind.  The partial sums of the two-stage reduction and the
 * results live in a fixed 16 MiB scratch array that the library keeps on every
 * device it runs on until the process ends (its address is looked up once per
 * device by qmg_create).  Limit: 2*nrhs + nrhs * ceil(12 V / 2048) * 2 <= 2^21
 * doubles (V lattice sites): 64x32^3 takes any nrhs <= 64, 64^4 nrhs <= 21;
 * larger requests return QMG_E_ARG.  Results are bitwise those of
 * qmg_field_dot (same kernels, same summation order).  Every call on one
 * device shares that device's scratch, so calls that overlap on one GPU (other
 * host threads, other contexts, other streams) race; synchronises the stream. */
qmg_status qmg_field_dot_noalloc(qmg_ctx* ctx, double* result, const void* a, const void* b, int nrhs,
                                 qmg_prec p, hipStream_t stream);

/* Gauge field (device, canonical complex128), bare mass m0 of eq. (2.5) and
 * clover coefficient csw.  Builds the clover term on the device (clover-leaf
 * field strength, traceless) and keeps F64/F32/BF16 copies.  Invalidates the
 * multigrid hierarchy. */
qmg_status qmg_set_gauge(qmg_ctx* ctx, const double* U_canon, double m0, double csw,
                         hipStream_t stream);

/* out_k = Q in_k = Gamma5 D in_k (eq. (2.5), Q = Gamma5 D). */
qmg_status qmg_apply_Q(qmg_ctx* ctx, void* out, const void* in, int nrhs, qmg_prec p,
                       hipStream_t stream);
/* out_k = (Q - tau_k I) in_k (eq. (1.1)); tau: host array of nrhs shifts. */
qmg_status qmg_apply_Q_shifted(qmg_ctx* ctx, void* out, const void* in, const double* tau,
                               int nrhs, qmg_prec p, hipStream_t stream);
/* out_k = (D - tau_k Gamma5) in_k, the Gamma5-preconditioned operator (eq. (3.7)). */
qmg_status qmg_apply_A(qmg_ctx* ctx, void* out, const void* in, const double* tau,
                       int nrhs, qmg_prec p, hipStream_t stream);

/* nsweep red-black SAP sweeps (Sec. 2) on (D - tau_k Gamma5) x_k = f_k,
 * updating x in place; each block solve is n_mr minimal-residual steps from
 * zero on the block-restricted operator; colour-0 blocks first. */
qmg_status qmg_sap_smooth(qmg_ctx* ctx, void* x, const void* f, const double* tau, int nrhs,
                          int nsweep, int n_mr, qmg_prec p, hipStream_t stream);

/* Build the interpolation P from ntv test vectors W (internal F64 fields):
 * per aggregate (block x chirality half) the restrictions of W are
 * orthonormalised (modified Gram-Schmidt twice, column order), then the
 * Galerkin coarse operator D_c = P^H D P (Sec. 2) is assembled.
 * Returns QMG_E_NUMERIC for locally rank-deficient W. */
qmg_status qmg_set_test_vectors(qmg_ctx* ctx, const void* W, int ntv, hipStream_t stream);
/* Adaptive setup (reading of the paper's setup parameters, Sec. 4 parameter
 * table: 24 test vectors, 6 setup iterations, 4 smoothing steps): smooth W0
 * with `smooth` FP64 SAP sweeps (n_mr minimal-residual steps per block) on
 * D w = 0 and normalise, then setup_iters-1 rounds of inverse iteration
 * w <- M(tau = 0) w, normalised, rebuilding P and D_c after each round; M is
 * the two-level V-cycle (coarse GMRES to coarse_tol, at most coarse_maxiter
 * steps, then `smooth` SAP sweeps) computed in precision `prec` (QMG_F64 for
 * parity with an FP64 reference, QMG_F32 or QMG_BF16 for speed: the vectors
 * only steer the multigrid's quality).  W0 (ntv internal F64 fields, device)
 * is overwritten with the final test vectors.  QMG_E_NUMERIC when a vector
 * vanishes or W is locally rank deficient.  Synchronous. */
qmg_status qmg_setup_mg(qmg_ctx* ctx, void* W0, int ntv, int setup_iters, int smooth,
                        int n_mr, int coarse_maxiter, double coarse_tol, qmg_prec prec,
                        hipStream_t stream);

/* y_k = P^H v_k and v_k = P y_k (Sec. 2, R = P^H). */
qmg_status qmg_restrict(qmg_ctx* ctx, void* yc, const void* v, int nrhs, qmg_prec p,
                        hipStream_t stream);
qmg_status qmg_prolong(qmg_ctx* ctx, void* v, const void* yc, int nrhs, qmg_prec p,
                       hipStream_t stream);
/* out_k = (D_c - tau_k Gamma5^c) in_k, Gamma5^c = diag(+I_ntv, -I_ntv) per coarse site. */
qmg_status qmg_apply_coarse(qmg_ctx* ctx, void* out, const void* in, const double* tau,
                            int nrhs, qmg_prec p, hipStream_t stream);
/* Coarse GMRES from zero on (D_c - tau_k Gamma5^c) y_k = r_k, for exactly
 * `iters` steps when tol <= 0, else until ||res|| <= tol ||r_k||. */
qmg_status qmg_coarse_solve(qmg_ctx* ctx, void* y, const void* r, const double* tau, int nrhs,
                            int iters, double tol, qmg_prec p, hipStream_t stream);
/* One V-cycle z_k = M r_k (no pre-smoothing, coarse solve, nu_post SAP sweeps). */
qmg_status qmg_vcycle(qmg_ctx* ctx, void* z, const void* r, const double* tau, int nrhs,
                      const qmg_params* params, hipStream_t stream);

/* Solve (Q - tau_k I) x_k = b_k for k < nrhs (internal F64 fields x, b) by
 * FGMRES on (D - tau_k Gamma5) x_k = Gamma5 b_k, from x = 0 (or from the
 * caller's x when params->x0 = 1), each right-hand side with its own Krylov
 * space; stats: host array of nrhs (may be NULL).
 * Columns that have converged when a restart cycle ends leave the batch (when
 * at most three quarters remain): later cycles run on the others only, in
 * library buffers, and every column's x is written back to its own slot.
 * Returns QMG_NOT_CONVERGED if some column missed tol within maxiter. */
qmg_status qmg_solve_shifted(qmg_ctx* ctx, void* x, const void* b, const double* tau, int nrhs,
                             const qmg_params* params, qmg_stats* stats, hipStream_t stream);

/* Gauge force of L = phi^H Q x (Wilson part; QMG_E_STATE when csw != 0):
 * dU[x][mu][a][b] = dL/dU_mu(x)_ab and dUbar = dL/d conj(U_mu(x)_ab), both
 * canonical complex128 device arrays; phi, x internal F64 fields. */
qmg_status qmg_gauge_force(qmg_ctx* ctx, double* dU, double* dUbar, const void* phi,
                           const void* x, hipStream_t stream);

/* ---- Third multigrid level.  The paper's solver (DD-alpha-AMG) is multilevel;
 * its experiments use two levels (eq. (2.8), Sec. 4).  A third level repeats
 * the first coarse level's construction (Sec. 2 aggregation, Sec. 3.1 P from
 * test vectors) on the block lattice: aggregates of block2 level-2 sites (the
 * lattice blocks), each split by coarse chirality, ntv2 test vectors per
 * aggregate orthonormalised (modified Gram-Schmidt, two passes per column),
 * Galerkin operator D3 = P2^H D_c P2 with self and 8 neighbour blocks.
 *
 * Level-2 vectors are the coarse vectors of qmg_restrict ([nrhs][nb][2 ntv],
 * internal site order of qmg_coarse_site_order); level-3 vectors are
 * [nrhs][n3][2 ntv2] with aggregates numbered lexicographically by aggregate
 * coordinate (X_mu / block2_mu for block coordinate X), components
 * [chirality +: j < ntv2, chirality -: j < ntv2].  Vectors are FP64 for
 * QMG_F64 and FP32 otherwise, like the coarse vectors.
 *
 * qmg_set_level3_vectors: W2 holds ntv2 FP64 level-2 vectors (device), used
 * as given.  block2 must divide the block lattice with >= 2 aggregates per
 * direction; 1 <= ntv2 <= 24 and ntv2 <= bs2 * ntv (bs2 level-2 sites per
 * aggregate, ntv components per chirality on level 2), bs2 * ntv <= 1024.  QMG_E_NUMERIC if the
 * vectors are locally rank deficient; QMG_E_STATE before P / D_c exist.  A
 * later rebuild of P / D_c (qmg_set_test_vectors, qmg_setup_mg, interpolation
 * updates of the eigensolver) drops the level.  Synchronous. */
qmg_status qmg_set_level3_vectors(qmg_ctx* ctx, const void* W2, int ntv2, const int block2[4],
                                  hipStream_t stream);
/* Setup of the level-2 test vectors (reading: the level-1 setup one level
 * down): W2 (in/out, ntv2 FP64 level-2 vectors, e.g. P^H w_j of the level-1
 * test vectors) is normalised, the level built, then setup_iters - 1 rounds of
 * inverse iteration w <- M2(tau = 0) w (FP64; M2 with l3_iters level-3 GMRES
 * steps and `smooth` level-2 GMRES smoothing steps), each normalised and
 * followed by a rebuild.  Synchronous. */
qmg_status qmg_setup_level3(qmg_ctx* ctx, void* W2, int ntv2, const int block2[4], int setup_iters, int smooth,
                            int l3_iters, hipStream_t stream);
/* y3 = P2^H y2 and y2 = P2 y3 (level-2 <-> level-3 vectors in the coarse precision of p). */
qmg_status qmg_restrict_l3(qmg_ctx* ctx, void* y3, const void* y2, int nrhs, qmg_prec p, hipStream_t stream);
qmg_status qmg_prolong_l3(qmg_ctx* ctx, void* y2, const void* y3, int nrhs, qmg_prec p, hipStream_t stream);
/* out_k = (D3 - tau_k Gamma5^cc) in_k on level-3 vectors (D3 stored FP64, or FP32 for
 * QMG_F32 / QMG_BF16). */
qmg_status qmg_apply_l3(qmg_ctx* ctx, void* out, const void* in, const double* tau, int nrhs, qmg_prec p,
                        hipStream_t stream);
/* The level-2 solve of a three-level V-cycle: k2 FGMRES steps from zero on
 * A_c(tau_k) y_k = r_k, right-preconditioned by the level-2 cycle M2 (k3 GMRES
 * steps on A3 from zero on P2^H r, prolongation, s2 GMRES smoothing steps on the
 * level-2 residual equation); every scalar stays on the device. */
qmg_status qmg_level2_solve(qmg_ctx* ctx, void* y, const void* r, const double* tau, int nrhs, int k2, int k3,
                            int s2, qmg_prec p, hipStream_t stream);
/* Level-3 size: number of aggregates (level-3 sites) and components per site; 0, 0 before a build. */
qmg_status qmg_level3_shape(const qmg_ctx* ctx, int* n3, int* nc3);

/* Local coherence measure lc(v_k) = ||Pi v_k|| / ||v_k|| (Sec. 3.1), Pi the
 * orthogonal projection on the range of the current interpolation P; v:
 * nrhs internal F64 fields; lc: host array [nrhs].  Since P has orthonormal
 * columns per aggregate, ||Pi v|| = ||P^H v||.  Needs qmg_set_test_vectors or
 * qmg_setup_mg; synchronises the stream. */
qmg_status qmg_local_coherence(qmg_ctx* ctx, double* lc, const void* v, int nrhs, hipStream_t stream);

/* ---- GD-lambdaAMG eigensolver (Alg. GD-lambdaAMG, Sec. 3.3; defaults from
 * the paper's parameter table, see qmg_default_eig_params). */
typedef struct {
  int m_min;           /* search-space size kept at a thick restart (30) */
  int m_max;           /* search-space size that triggers a restart (50) */
  double tol;          /* lock when ||Q u - theta u|| <= tol, ||u|| = 1 (1e-8) */
  int maxiter;         /* outer iterations (expansions) */
  double inner_tol;    /* correction-equation relative residual (0.1) */
  int inner_maxiter;   /* FGMRES iterations per correction equation (5) */
  int update_interp;   /* 1: rebuild P and D_c from the ntv converged eigenvectors
                          closest to the current target after each lock */
  int block;           /* targets per outer step (1..16): the correction equations of
                          the `block` unlocked harmonic Ritz pairs of smallest |theta|
                          are solved as one batched multi-shift solve and all of them
                          expand the space (1: one target per step, as Alg. GD-lambdaAMG) */
  qmg_params solve;    /* inner solver settings (precision, smoother, coarse steps);
                          tol, maxiter and use_graph are overridden */
  int extraction;      /* 0: harmonic Ritz pairs of the pencil (QV)^H (QV) s = theta (QV)^H V s
                          (Sec. 3.2, the method's choice for the eigenvalues of smallest
                          modulus); 1: Rayleigh-Ritz pairs V^H Q V s = theta s (the extraction
                          of the paper's Ritz versus harmonic Ritz comparison, Sec. 4) */
  int both_signs;      /* 1 (default): each step targets the `block` unlocked pairs of smallest
                          |theta| of each sign (2 block correction equations, one batched solve)
                          and thick restarts keep both signs alternately; needs
                          m_min + 2 block <= m_max.  0: one target per step, the unlocked pair of
                          smallest |theta|, restarts keep the m_min of smallest |theta|
                          (Alg. GD-lambdaAMG as printed), which on a nearly symmetric spectrum can
                          lock the smallest pairs of one sign only instead of the smallest |lambda| */
} qmg_eig_params;

typedef struct {
  int iters;           /* outer iterations (search-space expansions) */
  int converged;       /* eigenpairs locked */
  int inner_iters;     /* FGMRES iterations over all correction equations */
  int interp_updates;  /* interpolation rebuilds */
  double seconds;      /* wall time */
} qmg_eig_stats;

qmg_eig_params qmg_default_eig_params(void);

/* Eigenpairs of Q = Gamma5 D of smallest modulus by generalized Davidson with
 * harmonic Ritz extraction (the pencil (QV)^H (QV) s = theta (QV)^H V s),
 * locking, thick restarts and multigrid-preconditioned correction equations
 * (D - theta Gamma5) t = Gamma5 r (Alg. GD-lambdaAMG, Sec. 3.3).
 *   lambda: host array [nev], the Rayleigh quotients u^H Q u of the locked
 *           vectors, in the order they converged;
 *   X:      device, nev internal F64 fields (output, orthonormal);
 *   V0:     device, n0 internal F64 fields spanning the initial space (for
 *           example the test vectors of qmg_setup_mg; may be NULL with n0 = 0);
 *   t0:     device, one internal F64 field, the first expansion vector.
 * Needs qmg_set_gauge (and, for a two-level inner solver and interpolation
 * updates, qmg_set_test_vectors or qmg_setup_mg; for solve.levels = 3 also
 * qmg_set_level3_vectors / qmg_setup_level3: every interpolation update then
 * rebuilds the third level from P^H w_j of the first ntv2 new test vectors,
 * same aggregates).  Synchronises the stream.
 * Once nev pairs are locked the iteration goes on while the smallest unlocked
 * |theta| lies below the largest locked |lambda| by more than its residual; a
 * pair that then converges replaces that largest one.  Needs m_min + block <=
 * m_max and n0 + 1 <= m_max.
 * Returns QMG_NOT_CONVERGED when maxiter ends the run early (lambda and X hold
 * stats->converged pairs). */
qmg_status qmg_eigensolve(qmg_ctx* ctx, int nev, double* lambda, void* X, const void* V0, int n0,
                          const void* t0, const qmg_eig_params* params, qmg_eig_stats* stats,
                          hipStream_t stream);

/* Host-side dense Hermitian eigensolver used for the harmonic Ritz pencil
 * (cyclic Jacobi): a is m x m, column-major, interleaved re/im doubles; w gets
 * the eigenvalues in ascending order, z (m x m, same layout) the eigenvectors
 * as columns.  Pure host code (no device needed).  QMG_E_ARG on bad sizes. */
qmg_status qmg_hermitian_eig(int m, const double* a, double* w, double* z);

/* Time the launch variants of the hot kernels for this context's shape and
 * pick the fastest; results are cached in a JSON file keyed by device
 * architecture and lattice shape (path may be NULL: no file). */
qmg_status qmg_autotune(qmg_ctx* ctx, const char* cache_json_path);

/* Bandwidth probe (not part of the method): copies `bytes` (a multiple of 16,
 * both device pointers 16-byte aligned, regions not overlapping) from src to
 * dst with a plain streaming kernel on `stream`, the reference against which
 * the achieved bandwidth of the stencil kernels is read.  QMG_E_ARG on bad
 * sizes or alignment, QMG_E_HIP if the launch fails.  Needs no context. */
qmg_status qmg_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* QMG_H */
