// The C interface: context, validation, error reporting and dispatch to the
// kernel launchers and solver drivers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qmg_ctx.h"

// Scratch of qmg_field_dot_noalloc: the per-chunk partial sums of the
// two-stage dot products followed by the final results.  One copy per device
// (16 MiB), held until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns on that device, never through the name.
constexpr size_t kNoAllocDoubles = (size_t)1 << 21;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[256] = {};  // per device, filled once by the first qmg_create on that device

// device address of this device's scratch (device already current); nullptr on failure
double* scratch_address(int device) {
  if (device < 0 || device >= 256) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    double* ptr = nullptr;
    if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}
}  // namespace

qmg_status set_err(qmg_ctx* c, qmg_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

qmg_status hip_err(qmg_ctx* c, hipError_t e, const char* where) {
  if (e == hipErrorOutOfMemory) return set_err(c, QMG_E_NOMEM, std::string(where) + ": out of device memory");
  return set_err(c, QMG_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

size_t field_elems(const qmg_ctx* c) { return (size_t)c->g.V * 12; }
size_t coarse_elems(const qmg_ctx* c) { return (size_t)c->g.nb * 2 * c->ntv; }

void* ws_get(qmg_ctx* c, const std::string& name, size_t bytes) {
  auto it = c->ws.find(name);
  if (it != c->ws.end() && it->second.second >= bytes) return it->second.first;
  if (it != c->ws.end()) {
    hipDeviceSynchronize();
    hipFree(it->second.first);
    c->ws.erase(it);
    drop_graphs(c);  // captured graphs may hold the old address
  }
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
  c->ws[name] = {p, bytes};
  return p;
}

void ws_release(qmg_ctx* c, const std::string& name) {
  auto it = c->ws.find(name);
  if (it == c->ws.end()) return;
  hipDeviceSynchronize();
  hipFree(it->second.first);
  c->ws.erase(it);
  drop_graphs(c);
}

void drop_graphs(qmg_ctx* c) {
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  c->ws_epoch++;
}

namespace {

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

qmg_status check_prec(qmg_ctx* c, int p) {
  if (p != QMG_F64 && p != QMG_F32 && p != QMG_BF16) return set_err(c, QMG_E_ARG, "unknown precision");
  return QMG_OK;
}
qmg_status check_nrhs(qmg_ctx* c, int nrhs) {
  if (nrhs < 1 || nrhs > QMG_MAXRHS) return set_err(c, QMG_E_ARG, "nrhs must be in 1..64");
  return QMG_OK;
}
qmg_status need_gauge(qmg_ctx* c) {
  if (!c->have_gauge) return set_err(c, QMG_E_STATE, "qmg_set_gauge has not been called");
  return QMG_OK;
}
qmg_status need_sap(qmg_ctx* c) {
  if (!c->sap_ok)
    return set_err(c, QMG_E_ARG,
                   "SAP and multigrid need an even number (>= 2) of blocks per direction and 16..256 sites per block");
  return QMG_OK;
}
qmg_status need_mg(qmg_ctx* c) {
  if (!c->have_mg) return set_err(c, QMG_E_STATE, "qmg_set_test_vectors / qmg_setup_mg has not been called");
  return QMG_OK;
}
qmg_status check_tau(qmg_ctx* c, const double* tau, int nrhs) {
  if (!tau) return set_err(c, QMG_E_ARG, "tau is NULL");
  for (int k = 0; k < nrhs; ++k)
    if (!std::isfinite(tau[k])) return set_err(c, QMG_E_ARG, "tau must be finite");
  return QMG_OK;
}

// levels = 3 needs a built third level and sane step counts
qmg_status check_levels(qmg_ctx* c, const qmg_params& p) {
  if (p.levels != 2 && p.levels != 3) return set_err(c, QMG_E_ARG, "levels must be 2 or 3");
  if (p.levels == 3 && p.use_coarse) {
    if (p.l3_iters < 1 || p.l2_smooth < 0 || p.coarse_maxiter < 1)
      return set_err(c, QMG_E_ARG, "levels = 3: need l3_iters >= 1, l2_smooth >= 0, coarse_maxiter >= 1");
    if (!c->l3.ok) return set_err(c, QMG_E_STATE, "levels = 3: qmg_set_level3_vectors / qmg_setup_level3 has not been called");
  }
  return QMG_OK;
}

#define QMG_TRY(x)                  \
  do {                              \
    qmg_status _s = (x);            \
    if (_s != QMG_OK) return _s;    \
  } while (0)

qmg_status hipchk(qmg_ctx* c, hipError_t e, const char* where) {
  return e == hipSuccess ? QMG_OK : hip_err(c, e, where);
}

void free_ptr(void*& p) {
  if (p) hipFree(p);
  p = nullptr;
}

}  // namespace

qmg_status set_ds_order(qmg_ctx* c, int order) {
  if (order < 0 || order >= kNumDsOrders) return set_err(c, QMG_E_ARG, "stencil order");
  const Geom& g = c->g;
  int T[4];
  for (int mu = 0; mu < 4; ++mu) {
    T[mu] = std::min(kTileShapes[order][mu], g.nbk[mu]);
    while (g.nbk[mu] % T[mu] != 0) --T[mu];
  }
  std::vector<int> id_of_lex((size_t)g.nb);
  for (int b = 0; b < g.nb; ++b) id_of_lex[(size_t)c->lex_of_block[b]] = b;
  std::vector<int> tord;
  tord.reserve((size_t)g.nb);
  int nt[4];
  for (int mu = 0; mu < 4; ++mu) nt[mu] = g.nbk[mu] / T[mu];
  for (int t0 = 0; t0 < nt[0]; ++t0)
    for (int t1 = 0; t1 < nt[1]; ++t1)
      for (int t2 = 0; t2 < nt[2]; ++t2)
        for (int t3 = 0; t3 < nt[3]; ++t3)
          for (int i0 = 0; i0 < T[0]; ++i0)
            for (int i1 = 0; i1 < T[1]; ++i1)
              for (int i2 = 0; i2 < T[2]; ++i2)
                for (int i3 = 0; i3 < T[3]; ++i3) {
                  const int X[4] = {t0 * T[0] + i0, t1 * T[1] + i1, t2 * T[2] + i2, t3 * T[3] + i3};
                  const int lex = ((X[0] * g.nbk[1] + X[1]) * g.nbk[2] + X[2]) * g.nbk[3] + X[3];
                  tord.push_back(id_of_lex[(size_t)lex]);
                }
  std::vector<char> seen((size_t)g.nb, 0);
  for (int b : tord) {
    if (b < 0 || b >= g.nb || seen[(size_t)b]) return set_err(c, QMG_E_STATE, "stencil order is not a permutation");
    seen[(size_t)b] = 1;
  }
  if ((int)tord.size() != g.nb) return set_err(c, QMG_E_STATE, "stencil order is not a permutation");
  if (!c->d_tord && hipMalloc(&c->d_tord, sizeof(int) * (size_t)g.nb) != hipSuccess)
    return set_err(c, QMG_E_NOMEM, "stencil order table");
  hipError_t e = hipMemcpy(c->d_tord, tord.data(), sizeof(int) * (size_t)g.nb, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(c, e, "stencil order table");
  c->tile_blocks = T[0] * T[1] * T[2] * T[3];
  c->tune.ds_order = order;
  return QMG_OK;
}

extern "C" {

qmg_params qmg_default_params(void) {
  qmg_params p;
  p.tol = 1e-10;
  p.maxiter = 1000;
  p.restart = 16;
  p.nu_post = 3;
  p.n_mr = 3;
  p.coarse_maxiter = 50;
  p.coarse_tol = 0.5;
  p.mg_prec = QMG_F64;
  p.use_coarse = 1;
  p.use_graph = 0;
  p.q_form = 0;
  p.smoother = 0;
  p.levels = 2;
  p.l3_iters = 8;
  p.l2_smooth = 2;
  p.x0 = 0;
  return p;
}

qmg_eig_params qmg_default_eig_params(void) {
  qmg_eig_params e;
  e.m_min = 30;
  e.m_max = 50;
  e.tol = 1e-8;
  e.maxiter = 10000;
  e.inner_tol = 0.1;
  e.inner_maxiter = 5;
  e.update_interp = 1;
  e.block = 1;
  e.solve = qmg_default_params();
  e.solve.mg_prec = QMG_F32;
  e.solve.restart = 5;
  e.extraction = 0;
  e.both_signs = 1;
  return e;
}

qmg_status qmg_hermitian_eig(int m, const double* a, double* w, double* z) {
  if (m < 1 || m > 4096 || !a || !w || !z) return QMG_E_ARG;
  std::vector<std::complex<double>> A((size_t)m * m), Z;
  for (size_t i = 0; i < A.size(); ++i) A[i] = {a[2 * i], a[2 * i + 1]};
  std::vector<double> ev;
  herm_eig(m, A, ev, Z);
  for (int k = 0; k < m; ++k) w[k] = ev[k];
  for (size_t i = 0; i < Z.size(); ++i) {
    z[2 * i] = Z[i].real();
    z[2 * i + 1] = Z[i].imag();
  }
  return QMG_OK;
}

qmg_status qmg_create(qmg_ctx** out, const int dims[4], const int block[4], int device) {
  if (!out || !dims || !block) return QMG_E_ARG;
  *out = nullptr;
  qmg_ctx* c = new qmg_ctx();
  c->device = device;
  Geom& g = c->g;
  int64_t V = 1;
  int nb = 1, bs = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (dims[mu] < 1 || !is_pow2(block[mu]) || dims[mu] % block[mu]) {
      delete c;
      return QMG_E_ARG;
    }
    g.dims[mu] = dims[mu];
    g.block[mu] = block[mu];
    g.nbk[mu] = dims[mu] / block[mu];
    g.msk[mu] = block[mu] - 1;
    V *= dims[mu];
    nb *= g.nbk[mu];
    bs *= block[mu];
  }
  if (bs > 1024 || V > (int64_t)1 << 31 || (int64_t)nb * 36 * bs * 16 > ((int64_t)1 << 40)) {
    delete c;
    return QMG_E_ARG;
  }
  g.sh[3] = 0;
  g.sh[2] = ilog2(block[3]);
  g.sh[1] = g.sh[2] + ilog2(block[2]);
  g.sh[0] = g.sh[1] + ilog2(block[1]);
  g.bs_log = ilog2(bs);
  g.nb = nb;
  g.V = V;
  c->sap_ok = bs <= 256 && bs >= 16;
  for (int mu = 0; mu < 4; ++mu) c->sap_ok = c->sap_ok && g.nbk[mu] >= 2 && g.nbk[mu] % 2 == 0;
  // colour-major block numbering
  std::vector<int> id_of_lex(nb);
  c->lex_of_block.assign(nb, 0);
  int next = 0;
  for (int col = 0; col < 2; ++col)
    for (int lex = 0; lex < nb; ++lex) {
      int r = lex, X[4], sum = 0;
      for (int mu = 3; mu >= 0; --mu) { X[mu] = r % g.nbk[mu]; r /= g.nbk[mu]; sum += X[mu]; }
      if (sum % 2 != col) continue;
      id_of_lex[lex] = next;
      c->lex_of_block[next] = lex;
      ++next;
    }
  g.ncol0 = 0;
  c->h_bcoord.assign((size_t)nb * 4, 0);
  c->h_nbr.assign((size_t)nb * 8, 0);
  for (int b = 0; b < nb; ++b) {
    int r = (int)c->lex_of_block[b], X[4], sum = 0;
    for (int mu = 3; mu >= 0; --mu) { X[mu] = r % g.nbk[mu]; r /= g.nbk[mu]; sum += X[mu]; }
    if (sum % 2 == 0) ++g.ncol0;
    for (int mu = 0; mu < 4; ++mu) c->h_bcoord[b * 4 + mu] = X[mu];
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = 0; dir < 2; ++dir) {
        int Y[4] = {X[0], X[1], X[2], X[3]};
        Y[mu] = (Y[mu] + (dir == 0 ? 1 : g.nbk[mu] - 1)) % g.nbk[mu];
        int lex = ((Y[0] * g.nbk[1] + Y[1]) * g.nbk[2] + Y[2]) * g.nbk[3] + Y[3];
        c->h_nbr[b * 8 + 2 * mu + dir] = id_of_lex[lex];
      }
  }
  std::vector<int> lexord(id_of_lex);
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&c->d_nbr, sizeof(int) * nb * 8) != hipSuccess ||
      hipMalloc(&c->d_bcoord, sizeof(int) * nb * 4) != hipSuccess ||
      hipMalloc(&c->d_lexord, sizeof(int) * nb) != hipSuccess ||
      hipMemcpy(c->d_lexord, lexord.data(), sizeof(int) * nb, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_nbr, c->h_nbr.data(), sizeof(int) * nb * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_bcoord, c->h_bcoord.data(), sizeof(int) * nb * 4, hipMemcpyHostToDevice) != hipSuccess) {
    qmg_destroy(c);
    return QMG_E_HIP;
  }
  g.nbr = c->d_nbr;
  g.bcoord = c->d_bcoord;
  g.lexord = c->d_lexord;
  c->noalloc_scratch = scratch_address(device);
  if (!c->noalloc_scratch) {
    qmg_destroy(c);
    return QMG_E_HIP;
  }
  if (set_ds_order(c, c->tune.ds_order) != QMG_OK) {
    qmg_destroy(c);
    return QMG_E_HIP;
  }
  *out = c;
  return QMG_OK;
}


qmg_status qmg_destroy(qmg_ctx* c) {
  if (!c) return QMG_OK;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (int p = 0; p < 3; ++p) {
    free_ptr(c->U[p]);
    free_ptr(c->Dg[p]);
  }
  for (auto& kv : c->ws) hipFree(kv.second.first);
  if (c->d_nbr) hipFree(c->d_nbr);
  if (c->d_bcoord) hipFree(c->d_bcoord);
  if (c->d_lexord) hipFree(c->d_lexord);
  if (c->d_tord) hipFree(c->d_tord);
  delete c;
  return QMG_OK;
}

const char* qmg_last_error(const qmg_ctx* c) { return c ? c->err.c_str() : "null context"; }

size_t qmg_field_bytes(const qmg_ctx* c, qmg_prec p) { return c ? field_elems(c) * cbytes(p) : 0; }

size_t qmg_coarse_bytes(const qmg_ctx* c, qmg_prec p) {
  return c ? (size_t)c->g.nb * 2 * c->ntv * cbytes(coarse_prec(p)) : 0;
}

qmg_status qmg_coarse_site_order(const qmg_ctx* c, int64_t* out, int64_t n) {
  if (!c || !out || n < c->g.nb) return QMG_E_ARG;
  for (int b = 0; b < c->g.nb; ++b) out[b] = c->lex_of_block[b];
  return QMG_OK;
}

qmg_status qmg_pack(qmg_ctx* c, void* dev, const double* canon, int nrhs, qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  if (!dev || !canon || nrhs < 1) return set_err(c, QMG_E_ARG, "pack: bad arguments");
  hipSetDevice(c->device);
  return hipchk(c, launch_pack(c->g, dev, p, canon, nrhs, s), "pack");
}

qmg_status qmg_unpack(qmg_ctx* c, double* canon, const void* dev, int nrhs, qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  if (!dev || !canon || nrhs < 1) return set_err(c, QMG_E_ARG, "unpack: bad arguments");
  hipSetDevice(c->device);
  return hipchk(c, launch_unpack(c->g, canon, dev, p, nrhs, s), "unpack");
}

qmg_status qmg_field_dot(qmg_ctx* c, double* result, const void* a, const void* b, int nrhs, qmg_prec p,
                         hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  if (!result || !a || !b) return set_err(c, QMG_E_ARG, "field_dot: null pointer");
  hipSetDevice(c->device);
  const int64_t n = (int64_t)field_elems(c);
  double* d = (double*)ws_get(c, "dot_out", sizeof(double) * 2 * nrhs);
  double* part = (double*)ws_get(c, "dot_part", sizeof(double) * multidot_partial_doubles(n, 1, nrhs));
  if (!d || !part) return set_err(c, QMG_E_NOMEM, "field_dot: out of device memory");
  QMG_TRY(hipchk(c, launch_multidot(p, d, a, 0, 1, b, n, n, nrhs, part, s), "field_dot"));
  QMG_TRY(hipchk(c, hipMemcpyAsync(result, d, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s), "field_dot D2H"));
  return hipchk(c, hipStreamSynchronize(s), "field_dot sync");
}

qmg_status qmg_field_dot_noalloc(qmg_ctx* c, double* result, const void* a, const void* b, int nrhs, qmg_prec p,
                                 hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  if (!result || !a || !b) return set_err(c, QMG_E_ARG, "field_dot_noalloc: null pointer");
  const int64_t n = (int64_t)field_elems(c);
  const size_t need = 2 * (size_t)nrhs + multidot_partial_doubles(n, 1, nrhs);
  if (need > kNoAllocDoubles)
    return set_err(c, QMG_E_ARG, "field_dot_noalloc: nrhs x lattice volume exceeds the fixed scratch (" +
                                     std::to_string(need) + " > " + std::to_string(kNoAllocDoubles) + " doubles)");
  hipSetDevice(c->device);
  double* d = c->noalloc_scratch;
  double* part = d + 2 * (size_t)nrhs;
  QMG_TRY(hipchk(c, launch_multidot(p, d, a, 0, 1, b, n, n, nrhs, part, s), "field_dot_noalloc"));
  QMG_TRY(hipchk(c, hipMemcpyAsync(result, d, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s),
                 "field_dot_noalloc D2H"));
  return hipchk(c, hipStreamSynchronize(s), "field_dot_noalloc sync");
}

qmg_status qmg_set_gauge(qmg_ctx* c, const double* U, double m0, double csw, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  if (!U || !std::isfinite(m0) || !std::isfinite(csw)) return set_err(c, QMG_E_ARG, "set_gauge: bad arguments");
  hipSetDevice(c->device);
  const size_t nel = (size_t)c->g.nb * 36 * ((size_t)1 << c->g.bs_log);
  for (int p = 0; p < 3; ++p)
    if (!c->U[p] && hipMalloc(&c->U[p], nel * cbytes(p)) != hipSuccess)
      return set_err(c, QMG_E_NOMEM, "set_gauge: out of device memory");
  QMG_TRY(hipchk(c, launch_pack_gauge(c->g, c->U[QMG_F64], U, s), "pack gauge"));
  for (int p = 1; p < 3; ++p)
    QMG_TRY(hipchk(c, launch_convert(c->U[p], p, c->U[QMG_F64], QMG_F64, (int64_t)nel, s), "convert gauge"));
  c->clover = csw != 0.0;
  if (c->clover) {
    for (int p = 0; p < 3; ++p)
      if (!c->Dg[p] && hipMalloc(&c->Dg[p], nel * cbytes(p)) != hipSuccess)
        return set_err(c, QMG_E_NOMEM, "set_gauge: out of device memory");
    QMG_TRY(hipchk(c, launch_clover(c->g, c->Dg[QMG_F64], c->U[QMG_F64], m0, csw, s), "clover"));
    for (int p = 1; p < 3; ++p)
      QMG_TRY(hipchk(c, launch_convert(c->Dg[p], p, c->Dg[QMG_F64], QMG_F64, (int64_t)nel, s), "convert clover"));
  }
  QMG_TRY(hipchk(c, hipStreamSynchronize(s), "set_gauge sync"));
  c->m0 = m0;
  c->csw = csw;
  c->have_gauge = true;
  c->have_mg = false;
  drop_graphs(c);  // graphs carry m0 and the clover flag as kernel arguments
  return QMG_OK;
}

static qmg_status apply_common(qmg_ctx* c, void* out, const void* in, const double* tau, int nrhs, qmg_prec p,
                               int mode, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_gauge(c));
  if (!out || !in) return set_err(c, QMG_E_ARG, "apply: null field");
  if (out == in) return set_err(c, QMG_E_ARG, "apply: out and in must not alias");
  std::vector<double> t(nrhs, 0.0);
  if (tau) {
    QMG_TRY(check_tau(c, tau, nrhs));
    for (int k = 0; k < nrhs; ++k) t[k] = tau[k];
  }
  hipSetDevice(c->device);
  return hipchk(c, launch_dslash(c, p, out, in, t.data(), nrhs, mode, s), "apply");
}

qmg_status qmg_apply_Q(qmg_ctx* c, void* out, const void* in, int nrhs, qmg_prec p, hipStream_t s) {
  return apply_common(c, out, in, nullptr, nrhs, p, 1, s);
}

qmg_status qmg_apply_Q_shifted(qmg_ctx* c, void* out, const void* in, const double* tau, int nrhs, qmg_prec p,
                               hipStream_t s) {
  if (c && !tau) return set_err(c, QMG_E_ARG, "tau is NULL");
  return apply_common(c, out, in, tau, nrhs, p, 1, s);
}

qmg_status qmg_apply_A(qmg_ctx* c, void* out, const void* in, const double* tau, int nrhs, qmg_prec p,
                       hipStream_t s) {
  if (c && !tau) return set_err(c, QMG_E_ARG, "tau is NULL");
  return apply_common(c, out, in, tau, nrhs, p, 0, s);
}

qmg_status qmg_sap_smooth(qmg_ctx* c, void* x, const void* f, const double* tau, int nrhs, int nsweep, int n_mr,
                          qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_gauge(c));
  QMG_TRY(need_sap(c));
  QMG_TRY(check_tau(c, tau, nrhs));
  if (!x || !f || x == f || nsweep < 0 || n_mr < 0) return set_err(c, QMG_E_ARG, "sap_smooth: bad arguments");
  hipSetDevice(c->device);
  for (int sw = 0; sw < nsweep; ++sw)
    for (int col = 0; col < 2; ++col)
      QMG_TRY(hipchk(c, launch_sap_colour(c, p, x, f, tau, nrhs, col, n_mr, s), "sap"));
  return QMG_OK;
}

qmg_status qmg_set_test_vectors(qmg_ctx* c, const void* W, int ntv, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(need_gauge(c));
  QMG_TRY(need_sap(c));
  if (!W || ntv < 1 || ntv > 32) return set_err(c, QMG_E_ARG, "set_test_vectors: need 1 <= ntv <= 32");
  if (6 * ((int64_t)1 << c->g.bs_log) < ntv) return set_err(c, QMG_E_ARG, "ntv exceeds the aggregate size");
  hipSetDevice(c->device);
  return build_mg(c, W, ntv, s);
}

qmg_status qmg_setup_mg(qmg_ctx* c, void* W0, int ntv, int setup_iters, int smooth, int n_mr, int coarse_maxiter,
                        double coarse_tol, qmg_prec prec, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(need_gauge(c));
  QMG_TRY(need_sap(c));
  QMG_TRY(check_prec(c, prec));
  if (!W0 || ntv < 1 || ntv > 32 || setup_iters < 1 || smooth < 0 || n_mr < 0 || coarse_maxiter < 1)
    return set_err(c, QMG_E_ARG, "setup_mg: bad arguments");
  hipSetDevice(c->device);
  return solver_setup(c, W0, ntv, setup_iters, smooth, n_mr, coarse_maxiter, coarse_tol, prec, s);
}

qmg_status qmg_restrict(qmg_ctx* c, void* yc, const void* v, int nrhs, qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_mg(c));
  if (!yc || !v) return set_err(c, QMG_E_ARG, "restrict: null pointer");
  hipSetDevice(c->device);
  return hipchk(c, launch_restrict(c, p, yc, v, nrhs, s), "restrict");
}

qmg_status qmg_prolong(qmg_ctx* c, void* v, const void* yc, int nrhs, qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_mg(c));
  if (!yc || !v) return set_err(c, QMG_E_ARG, "prolong: null pointer");
  hipSetDevice(c->device);
  return hipchk(c, launch_prolong(c, p, v, yc, nrhs, s), "prolong");
}

qmg_status qmg_apply_coarse(qmg_ctx* c, void* out, const void* in, const double* tau, int nrhs, qmg_prec p,
                            hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_mg(c));
  QMG_TRY(check_tau(c, tau, nrhs));
  if (!out || !in || out == in) return set_err(c, QMG_E_ARG, "apply_coarse: bad pointers");
  hipSetDevice(c->device);
  return hipchk(c, launch_coarse_apply(c, p, out, in, tau, nrhs, s), "apply_coarse");
}

qmg_status qmg_coarse_solve(qmg_ctx* c, void* y, const void* r, const double* tau, int nrhs, int iters, double tol,
                            qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_mg(c));
  QMG_TRY(check_tau(c, tau, nrhs));
  if (!y || !r || y == r || iters < 1) return set_err(c, QMG_E_ARG, "coarse_solve: bad arguments");
  hipSetDevice(c->device);
  return solver_coarse_gmres(c, p, y, r, tau, nrhs, iters, tol, nullptr, s);
}

// ---- third level
static qmg_status check_block2(qmg_ctx* c, int ntv2, const int* block2) {
  if (!block2 || ntv2 < 1 || ntv2 > 24) return set_err(c, QMG_E_ARG, "level 3: need 1 <= ntv2 <= 24");
  int bs2 = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (block2[mu] < 1 || c->g.nbk[mu] % block2[mu] || c->g.nbk[mu] / block2[mu] < 2)
      return set_err(c, QMG_E_ARG, "level 3: block2 must divide the block lattice with >= 2 aggregates per direction");
    bs2 *= block2[mu];
  }
  if ((int64_t)bs2 * c->ntv > 1024) return set_err(c, QMG_E_ARG, "level 3: bs2 * ntv must be <= 1024");
  if (ntv2 > bs2 * c->ntv) return set_err(c, QMG_E_ARG, "level 3: ntv2 exceeds the aggregate size");
  return QMG_OK;
}

static qmg_status need_l3(qmg_ctx* c) {
  QMG_TRY(need_mg(c));
  if (!c->l3.ok) return set_err(c, QMG_E_STATE, "qmg_set_level3_vectors / qmg_setup_level3 has not been called");
  return QMG_OK;
}

qmg_status qmg_set_level3_vectors(qmg_ctx* c, const void* W2, int ntv2, const int block2[4], hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(need_mg(c));
  if (!W2) return set_err(c, QMG_E_ARG, "set_level3_vectors: null pointer");
  QMG_TRY(check_block2(c, ntv2, block2));
  hipSetDevice(c->device);
  return build_l3(c, W2, ntv2, block2, s);
}

qmg_status qmg_setup_level3(qmg_ctx* c, void* W2, int ntv2, const int block2[4], int setup_iters, int smooth,
                            int l3_iters, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(need_mg(c));
  if (!W2 || setup_iters < 1 || smooth < 0 || l3_iters < 1) return set_err(c, QMG_E_ARG, "setup_level3: bad arguments");
  QMG_TRY(check_block2(c, ntv2, block2));
  hipSetDevice(c->device);
  return solver_setup_l3(c, W2, ntv2, block2, setup_iters, smooth, l3_iters, s);
}

qmg_status qmg_restrict_l3(qmg_ctx* c, void* y3, const void* y2, int nrhs, qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_l3(c));
  if (!y3 || !y2) return set_err(c, QMG_E_ARG, "restrict_l3: null pointer");
  hipSetDevice(c->device);
  return hipchk(c, launch_restrict_l3(c, p, y3, y2, nrhs, s), "restrict_l3");
}

qmg_status qmg_prolong_l3(qmg_ctx* c, void* y2, const void* y3, int nrhs, qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_l3(c));
  if (!y3 || !y2) return set_err(c, QMG_E_ARG, "prolong_l3: null pointer");
  hipSetDevice(c->device);
  return hipchk(c, launch_prolong_l3(c, p, y2, y3, nrhs, s), "prolong_l3");
}

qmg_status qmg_apply_l3(qmg_ctx* c, void* out, const void* in, const double* tau, int nrhs, qmg_prec p,
                        hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_l3(c));
  QMG_TRY(check_tau(c, tau, nrhs));
  if (!out || !in || out == in) return set_err(c, QMG_E_ARG, "apply_l3: bad pointers");
  hipSetDevice(c->device);
  return hipchk(c, launch_apply_l3(c, p, out, in, tau, nrhs, s), "apply_l3");
}

qmg_status qmg_level2_solve(qmg_ctx* c, void* y, const void* r, const double* tau, int nrhs, int k2, int k3, int s2,
                            qmg_prec p, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_prec(c, p));
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_l3(c));
  QMG_TRY(check_tau(c, tau, nrhs));
  if (!y || !r || y == r || k2 < 1 || k3 < 1 || s2 < 0) return set_err(c, QMG_E_ARG, "level2_solve: bad arguments");
  hipSetDevice(c->device);
  return level2_kcycle(c, p, y, r, tau, nrhs, k2, k3, s2, s);
}

qmg_status qmg_level3_shape(const qmg_ctx* c, int* n3, int* nc3) {
  if (!c || !n3 || !nc3) return QMG_E_ARG;
  *n3 = c->l3.ok ? c->l3.n3 : 0;
  *nc3 = c->l3.ok ? 2 * c->l3.ntv2 : 0;
  return QMG_OK;
}

qmg_status qmg_vcycle(qmg_ctx* c, void* z, const void* r, const double* tau, int nrhs, const qmg_params* prm,
                      hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_gauge(c));
  QMG_TRY(need_sap(c));
  QMG_TRY(check_tau(c, tau, nrhs));
  if (!z || !r || z == r || !prm || prm->q_form < 0 || prm->q_form > 1 || prm->smoother < 0 || prm->smoother > 1)
    return set_err(c, QMG_E_ARG, "vcycle: bad arguments");
  QMG_TRY(check_prec(c, prm->mg_prec));
  if (prm->use_coarse) QMG_TRY(need_mg(c));
  QMG_TRY(check_levels(c, *prm));
  hipSetDevice(c->device);
  return solver_vcycle(c, z, r, tau, nrhs, prm, nullptr, s);
}

qmg_status qmg_solve_shifted(qmg_ctx* c, void* x, const void* b, const double* tau, int nrhs, const qmg_params* prm,
                             qmg_stats* st, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_gauge(c));
  QMG_TRY(need_sap(c));
  QMG_TRY(check_tau(c, tau, nrhs));
  if (!x || !b || x == b) return set_err(c, QMG_E_ARG, "solve_shifted: bad pointers");
  qmg_params prm0 = prm ? *prm : qmg_default_params();
  QMG_TRY(check_prec(c, prm0.mg_prec));
  if (!(prm0.tol > 0) || prm0.maxiter < 1 || prm0.restart < 1 || prm0.nu_post < 0 || prm0.n_mr < 0 ||
      prm0.coarse_maxiter < 1 || prm0.q_form < 0 || prm0.q_form > 1 || prm0.smoother < 0 || prm0.smoother > 1 ||
      prm0.x0 < 0 || prm0.x0 > 1)
    return set_err(c, QMG_E_ARG, "solve_shifted: bad parameters");
  QMG_TRY(check_levels(c, prm0));
  if (prm0.use_coarse) QMG_TRY(need_mg(c));
  hipSetDevice(c->device);
  return solver_fgmres(c, x, b, tau, nrhs, &prm0, st, s);
}

qmg_status qmg_gauge_force(qmg_ctx* c, double* dU, double* dUbar, const void* phi, const void* x, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(need_gauge(c));
  if (c->clover) return set_err(c, QMG_E_STATE, "gauge_force: only the Wilson part (csw = 0) is implemented");
  if (!dU || !dUbar || !phi || !x) return set_err(c, QMG_E_ARG, "gauge_force: null pointer");
  hipSetDevice(c->device);
  return hipchk(c, launch_force(c, dU, dUbar, phi, x, s), "gauge_force");
}

qmg_status qmg_local_coherence(qmg_ctx* c, double* lc, const void* v, int nrhs, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(check_nrhs(c, nrhs));
  QMG_TRY(need_mg(c));
  if (!lc || !v) return set_err(c, QMG_E_ARG, "local_coherence: null pointer");
  hipSetDevice(c->device);
  const int64_t nf = (int64_t)field_elems(c), ncs = (int64_t)coarse_elems(c);
  void* y = ws_get(c, "lc_y", (size_t)ncs * nrhs * 16);
  double* d = (double*)ws_get(c, "lc_d", sizeof(double) * 4 * nrhs);
  double* part = (double*)ws_get(c, "lc_part",
                                 sizeof(double) * std::max(multidot_partial_doubles(nf, 1, nrhs),
                                                           multidot_partial_doubles(ncs, 1, nrhs)));
  if (!y || !d || !part) return set_err(c, QMG_E_NOMEM, "out of device memory (local coherence)");
  hipError_t e = launch_restrict(c, QMG_F64, y, v, nrhs, s);
  // ||P^H v_k||^2 and ||v_k||^2 (squared norms as self dot products)
  if (e == hipSuccess) e = launch_multidot(QMG_F64, d, y, 0, 1, y, ncs, ncs, nrhs, part, s, 0);
  std::vector<double> hy(2 * nrhs), hv(2 * nrhs);
  if (e == hipSuccess) e = hipMemcpyAsync(hy.data(), d, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = launch_multidot(QMG_F64, d, v, 0, 1, v, nf, nf, nrhs, part, s, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(hv.data(), d, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "local coherence");
  for (int k = 0; k < nrhs; ++k) {
    if (!(hv[2 * k] > 0) || !std::isfinite(hv[2 * k]) || !std::isfinite(hy[2 * k]))
      return set_err(c, QMG_E_NUMERIC, "local coherence of a zero or non-finite vector");
    lc[k] = std::sqrt(std::max(0.0, hy[2 * k]) / hv[2 * k]);
  }
  return QMG_OK;
}

qmg_status qmg_eigensolve(qmg_ctx* c, int nev, double* lambda, void* X, const void* V0, int n0, const void* t0,
                          const qmg_eig_params* prm, qmg_eig_stats* st, hipStream_t s) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(need_gauge(c));
  QMG_TRY(need_sap(c));
  const qmg_eig_params p = prm ? *prm : qmg_default_eig_params();
  if (nev < 1 || !lambda || !X || !t0 || n0 < 0 || (n0 > 0 && !V0))
    return set_err(c, QMG_E_ARG, "eigensolve: bad arguments");
  if (p.m_max < 2 || p.m_min < 1 || p.block < 1 || p.block > 16 || p.both_signs < 0 || p.both_signs > 1 ||
      p.m_min + (p.both_signs ? 2 : 1) * p.block > p.m_max || n0 >= p.m_max ||
      !(p.tol > 0) || p.maxiter < 1 || !(p.inner_tol > 0) || p.inner_maxiter < 1 || p.extraction < 0 ||
      p.extraction > 1)
    return set_err(c, QMG_E_ARG, "eigensolve: bad parameters");
  QMG_TRY(check_prec(c, p.solve.mg_prec));
  if (p.solve.use_coarse) QMG_TRY(need_mg(c));
  QMG_TRY(check_levels(c, p.solve));
  hipSetDevice(c->device);
  return solver_eigensolve(c, nev, lambda, X, V0, n0, t0, &p, st, s);
}

qmg_status qmg_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (!dst || !src || bytes % 16 != 0 || (uintptr_t)dst % 16 != 0 || (uintptr_t)src % 16 != 0) return QMG_E_ARG;
  return launch_stream_copy(dst, src, bytes, s) == hipSuccess ? QMG_OK : QMG_E_HIP;
}

qmg_status qmg_autotune(qmg_ctx* c, const char* path) {
  if (!c) return QMG_E_ARG;
  QMG_TRY(need_gauge(c));
  hipSetDevice(c->device);
  return tune_run(c, path);
}

}  // extern "C"
