// Host-side context and the launchers each kernel file provides.
#pragma once
#include <hip/hip_runtime.h>
#include <complex>
#include <map>
#include <string>
#include <vector>

#include "../../include/qmg.h"
#include "qmg_device.h"

#define QMG_MAXRHS 64

// size in bytes of one complex number in storage precision p
inline size_t cbytes(int p) { return p == QMG_F64 ? 16 : (p == QMG_F32 ? 8 : 4); }
// coarse vectors are double for F64 and float otherwise
inline int coarse_prec(int p) { return p == QMG_F64 ? QMG_F64 : QMG_F32; }

// Stencil launch variants for 4^4 blocks: R right-hand sides per thread and a
// waves-per-SIMD occupancy target W (0: compiler's choice).  Variant 0 is the
// generic kernel (any block shape).
struct DsVariant { int R, W; };
// variants 8..10 walk all rhs groups of a block inside one work-group
// variant 11 is variant 1 writing its output with non-temporal stores
constexpr DsVariant kDsVariants[] = {{0, 0}, {1, 0}, {1, 2}, {1, 3}, {1, 4}, {2, 0}, {2, 2}, {4, 0},
                                     {1, 2}, {2, 0}, {2, 2}, {1, 0}};
constexpr int kNumDsVariants = 12;
// tiles of blocks (extent per direction, clamped to a divisor of the block grid)
constexpr int kTileShapes[][4] = {{1, 1, 1, 1}, {2, 2, 2, 2}, {2, 2, 2, 4}, {2, 2, 4, 4},
                                  {1, 2, 4, 8}, {2, 2, 4, 8}, {1, 1, 2, 8}, {1, 2, 2, 4}};
constexpr int kNumDsOrders = 8;

struct Tune {
  int dslash[3][2] = {{1, 1}, {1, 1}, {1, 1}};  // [prec][nrhs == 1 ? 0 : 1] -> variant index
  int dslash_xcd_remap = 1;                      // XCD-aware mapping of work-groups to blocks
  int force_variant = -1;                        // >= 0: use this stencil variant (tuning, tests)
  int sap_variant = 2;  // 0 generic SAP; 1, 2: LDS-staged 4^4 SAP (FP32 / BF16) with 1 or 2 rhs per work-group
  int coarse_rhs_tile = 4;                       // right-hand sides per coarse-apply work-group
  int coarse_mfma = 1;                           // MFMA coarse apply for many right-hand sides
  int transfer_mr = 1;                           // restrict / prolong kernels sharing P loads across rhs
  int restrict_mfma_min_rhs = 4;                 // restriction on MFMA from this many rhs (1000: never)
  int ds_order = 0;  // stencil work order: 0 blocks in lexicographic order, each with its rhs groups back to
                     // back; t > 0 tiles of kTileShapes[t] blocks, each tile's rhs groups back to back
  int coarse_mfma_min_rhs = 4;                   // smallest batch that takes the MFMA path
  bool tuned = false;
};

// Third multigrid level: aggregates of block2 level-2 sites (lattice blocks),
// ntv2 level-3 components per chirality.  Tables and operators live in the
// workspace; the level is dropped whenever P / D_c are rebuilt.
struct Level3 {
  bool ok = false;
  int ntv2 = 0, n3 = 0, bs2 = 0;
  int block2[4] = {0, 0, 0, 0};
  int dims3[4] = {0, 0, 0, 0};
  const int* sites = nullptr;  // [n3][bs2] level-2 site ids, lexicographic inside the aggregate
  const int* agg = nullptr;    // [nb] aggregate of each level-2 site
  const int* qloc = nullptr;   // [nb] index of the site inside its aggregate
  const int* keep = nullptr;   // [nb][9] 1 where stencil entry d of the site stays in its aggregate
  const int* nbr3 = nullptr;   // [n3][8] level-3 neighbours: 2 mu forward, 2 mu + 1 backward
  void* P2[2] = {nullptr, nullptr};  // F64, F32: [n3][2][bs2 * ntv][ntv2]
  void* D3[2] = {nullptr, nullptr};  // F64, F32: [n3][9][2 ntv2][2 ntv2] (transposed blocks)
};

struct qmg_ctx {
  int device = 0;
  Geom g{};                    // device pointers for tables inside
  int* d_nbr = nullptr;
  int* d_bcoord = nullptr;
  int* d_lexord = nullptr;
  int* d_tord = nullptr;       // block ids in stencil work order (tiles of tile_blocks blocks)
  int tile_blocks = 1;
  std::vector<int> h_nbr, h_bcoord;
  std::vector<int64_t> lex_of_block;
  bool sap_ok = false;
  // gauge
  bool have_gauge = false;
  double m0 = 0, csw = 0;
  bool clover = false;
  void* U[3] = {nullptr, nullptr, nullptr};
  void* Dg[3] = {nullptr, nullptr, nullptr};
  // multigrid
  bool have_mg = false;
  int ntv = 0;
  void* P[3] = {nullptr, nullptr, nullptr};
  void* Dc[3] = {nullptr, nullptr, nullptr};
  Level3 l3;
  // workspace
  std::map<std::string, std::pair<void*, size_t>> ws;
  std::map<std::string, std::vector<double>> hbuf;  // host staging for small Krylov data
  std::string err;
  Tune tune;
  std::map<std::string, hipGraphExec_t> graphs;  // captured V-cycles by (buffers, shifts, parameters)
  uint64_t ws_epoch = 0;                          // bumped whenever a workspace buffer moves
  hipStream_t cap_stream = nullptr;               // library stream used only to record graphs
  double* noalloc_scratch = nullptr;              // device address of this device's no-allocation scratch
};

size_t field_elems(const qmg_ctx* c);   // complex elements in one fine field
size_t coarse_elems(const qmg_ctx* c);  // complex elements in one coarse vector
size_t l3_elems(const qmg_ctx* c);      // complex elements in one level-3 vector

// stencil work order (tile shape index into kTileShapes); synchronous, not for use under capture
qmg_status set_ds_order(qmg_ctx* c, int order);

// named, lazily grown device workspace (never shrinks; freed by qmg_destroy)
void* ws_get(qmg_ctx* c, const std::string& name, size_t bytes);
void ws_release(qmg_ctx* c, const std::string& name);
void drop_graphs(qmg_ctx* c);

// ---- layout.hip
hipError_t launch_pack(const Geom& g, void* out, int p, const double* canon, int nrhs, hipStream_t s);
hipError_t launch_unpack(const Geom& g, double* canon, const void* in, int p, int nrhs, hipStream_t s);
hipError_t launch_convert(void* dst, int pd, const void* src, int ps, int64_t n, hipStream_t s);
// ---- gauge.hip
hipError_t launch_pack_gauge(const Geom& g, void* U64, const double* canon, hipStream_t s);
hipError_t launch_clover(const Geom& g, void* diag64, const void* U64, double m0, double csw,
                         hipStream_t s);
// ---- dslash.hip   mode 0: (D - tau Gamma5), mode 1: (Gamma5 D - tau)
hipError_t launch_dslash(const qmg_ctx* c, int p, void* out, const void* in, const double* tau,
                         int nrhs, int mode, hipStream_t s);
// (D - tau Gamma5) in FP64 arithmetic and storage, reading an input field stored in in_prec
hipError_t launch_dslash_d_in(const qmg_ctx* c, void* out, const void* in, int in_prec, const double* tau,
                              int nrhs, hipStream_t s, int mode = 0);
// ---- sap.hip
// qform: SAP for Q - tau = Gamma5 A_tau itself instead of A_tau
hipError_t launch_sap_colour(const qmg_ctx* c, int p, void* x, const void* f, const double* tau,
                             int nrhs, int colour, int n_mr, hipStream_t s, int qform = 0);
// ---- transfer.hip
hipError_t launch_build_P(const qmg_ctx* c, void* P64, const void* W, int ntv, int* d_fail,
                          hipStream_t s);
hipError_t launch_restrict(const qmg_ctx* c, int p, void* yc, const void* v, int nrhs, hipStream_t s);
hipError_t launch_prolong(const qmg_ctx* c, int p, void* v, const void* yc, int nrhs, hipStream_t s);
// ---- coarse.hip
hipError_t launch_split_stencil(const qmg_ctx* c, void* out9, const void* in, hipStream_t s);
// DcT[b][d][c0 + kk][:] = part[kk * 9 + d][b][:] for kk < kb (restricted parts, FP64)
hipError_t launch_scatter_dc(const qmg_ctx* c, void* Dc64, const void* part, int c0, int kb, hipStream_t s);
hipError_t launch_coarse_apply(const qmg_ctx* c, int p, void* out, const void* in, const double* tau,
                               int nrhs, hipStream_t s, int qform = 0);  // tau: host array
// level-3 operator A3(tau) = D3 - tau Gamma5^cc on level-3 vectors of the coarse precision of p
hipError_t launch_apply_l3(const qmg_ctx* c, int p, void* out, const void* in, const double* tau, int nrhs,
                           hipStream_t s, int qform = 0);
// ---- level3.hip (level-2 and level-3 vectors in the coarse precision of p)
qmg_status build_l3(qmg_ctx* c, const void* W2, int ntv2, const int block2[4], hipStream_t s);
hipError_t launch_restrict_l3(const qmg_ctx* c, int p, void* y3, const void* y2, int nrhs, hipStream_t s);
hipError_t launch_prolong_l3(const qmg_ctx* c, int p, void* y2, const void* y3, int nrhs, hipStream_t s);
qmg_status solver_setup_l3(qmg_ctx* c, void* W2, int ntv2, const int block2[4], int iters, int s2, int k3,
                           hipStream_t s);
// ---- blas.hip (vectors of n complex per right-hand side, k-th rhs at offset k*stride)
// dots[k*J + j] = <V_j,k , w_k> for j < J (V_j at base + j*vstride), FP64 results on device
hipError_t launch_multidot(int p, double* dots, const void* V, int64_t vstride, int J, const void* w,
                           int64_t n, int64_t stride, int nrhs, double* partial, hipStream_t s, int with_self = 0);
// w_k += sum_j coef[k*J + j] V_j,k and norms[2k] = ||w_k||^2 of the result; with copy
// (p == QMG_F64 only) the result is also written there in copy_prec (FP32 or BF16),
// bit for bit what launch_convert would write
hipError_t launch_axpy_norm(int p, void* w, const void* V, int64_t vstride, int J, const double* coef, int64_t n,
                            int64_t stride, int nrhs, double* norms, double* partial, hipStream_t s,
                            void* copy = nullptr, int copy_prec = QMG_F64);
// w_k += sum_j coef[k*J + j] * V_j,k   (coef complex double on device)
hipError_t launch_multiaxpy(int p, void* w, const void* V, int64_t vstride, int J, const double* coef,
                            int64_t n, int64_t stride, int nrhs, hipStream_t s);
// as launch_multiaxpy with w in FP64 and the J vectors V stored in vprec
hipError_t launch_multiaxpy_d(void* w, const void* V, int vprec, int64_t vstride, int J, const double* coef,
                              int64_t n, int64_t stride, int nrhs, hipStream_t s);
// y_k = a_k * x_k (a complex double on device, may alias); with copy (p == QMG_F64
// only) the result is also written there in copy_prec, as launch_convert would write it
hipError_t launch_scale(int p, void* y, const void* x, const double* a, int64_t n, int64_t stride,
                        int nrhs, hipStream_t s, void* copy = nullptr, int copy_prec = QMG_F64);
// y_k = x_k - y_k  (xmy) or y_k = y_k + x_k
hipError_t launch_xmy(int p, void* y, const void* x, int64_t n, int64_t stride, int nrhs, hipStream_t s);
hipError_t launch_gamma5_bs(int p, void* y, const void* x, int64_t n, int bs_log, hipStream_t s);
size_t multidot_partial_doubles(int64_t n, int J, int nrhs);
hipError_t launch_multidot_shared(int p, double* dots, const void* V, int64_t vstride, int J, const void* w,
                                  int64_t wstride, int nw, int64_t n, double* partial, hipStream_t s);
hipError_t launch_fill_zero(void* y, size_t bytes, hipStream_t s);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// ---- force.hip
hipError_t launch_unit_coarse(void* y, int nb, int nc, int col, hipStream_t s);
hipError_t launch_force(const qmg_ctx* c, double* dU, double* dUb, const void* phi, const void* x,
                        hipStream_t s);

// ---- solver.hip
qmg_status solver_coarse_gmres(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs,
                               int iters, double tol, int* iters_done, hipStream_t s, int qform = 0);
qmg_status coarse_gmres_device(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs, int iters,
                               hipStream_t s, int qform = 0);
// fixed-step device GMRES from zero on the fine stencil in precision p (smoother)
qmg_status fine_gmres_device(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs, int iters,
                             hipStream_t s, int qform = 0);
// the level-2 cycle M2 (level-3 GMRES correction, level-2 GMRES smoothing) and
// k2 steps of level-2 FGMRES preconditioned by it
qmg_status level2_cycle(qmg_ctx* c, int p, void* z, const void* r, const double* tau, int nrhs, int k3, int s2,
                        hipStream_t s, int qform = 0);
qmg_status level2_kcycle(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs, int k2, int k3,
                         int s2, hipStream_t s, int qform = 0);
// y += x for nrhs fields (n complex each, stride between fields)
hipError_t launch_add(int p, void* y, const void* x, int64_t n, int64_t stride, int nrhs, hipStream_t s);
// z = M r; z is written in precision zprec (FP64, or the preconditioner's own precision);
// r is read in precision rprec (FP64, or the preconditioner's own precision)
qmg_status solver_vcycle(qmg_ctx* c, void* z, const void* r, const double* tau, int nrhs,
                         const qmg_params* prm, int* coarse_iters, hipStream_t s, int zprec = QMG_F64,
                         int rprec = QMG_F64);
qmg_status solver_eigensolve(qmg_ctx* c, int nev, double* lambda, void* X, const void* V0, int n0,
                             const void* t0, const qmg_eig_params* prm, qmg_eig_stats* stats, hipStream_t s);
void herm_eig(int m, std::vector<std::complex<double>> a, std::vector<double>& w,
              std::vector<std::complex<double>>& z);
qmg_status solver_fgmres(qmg_ctx* c, void* x, const void* b, const double* tau, int nrhs,
                         const qmg_params* prm, qmg_stats* st, hipStream_t s);
qmg_status build_mg(qmg_ctx* c, const void* W, int ntv, hipStream_t s);
qmg_status solver_setup(qmg_ctx* c, void* W, int ntv, int iters, int smooth, int n_mr, int kc,
                        double ctol, int prec, hipStream_t s);
qmg_status tune_run(qmg_ctx* c, const char* path);

qmg_status set_err(qmg_ctx* c, qmg_status st, const std::string& msg);
qmg_status hip_err(qmg_ctx* c, hipError_t e, const char* where);
