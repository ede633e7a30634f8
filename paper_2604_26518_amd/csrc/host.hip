// Host runtime of libgmt: hierarchy construction, element constants, the
// pinned coarsest factorisation, V-cycle / PCG orchestration and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "common.h"

namespace gmt {

// ================================================================ errors

static thread_local std::string g_last_error;

void fail(gmt_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Failure{st, std::string(buf)};
}

template <typename F>
static gmt_status guarded(F&& fn) {
  try {
    fn();
    return GMT_OK;
  } catch (const Failure& f) {
    g_last_error = f.msg;
    return f.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return GMT_E_NOMEM;
  } catch (...) {
    g_last_error = "unknown internal error";
    return GMT_E_STATE;
  }
}

// ================================================================ allocation

void* Hier::raw_alloc(size_t bytes) {
  void* ptr = nullptr;
  const bool callback = p.alloc && !local_alloc;
  if (callback) {
    ptr = p.alloc(bytes, p.alloc_ctx);
    if (!ptr) fail(GMT_E_NOMEM, "allocator callback returned NULL for %zu bytes", bytes);
    owned.push_back(ptr);
  } else {
    hipError_t e = hipMalloc(&ptr, bytes);
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      fail(GMT_E_NOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    owned_hip.push_back(ptr);
  }
  return ptr;
}

void Hier::release(void* q) {
  auto it = std::find(owned.begin(), owned.end(), q);
  if (it != owned.end()) {
    owned.erase(it);
    if (p.release) p.release(q, p.alloc_ctx);
    return;
  }
  auto jt = std::find(owned_hip.begin(), owned_hip.end(), q);
  if (jt != owned_hip.end()) {
    owned_hip.erase(jt);
    (void)hipFree(q);
  }
}

void Hier::release_graphs() {
  for (PcgGraphs* g : {&g32, &g64, &gmx}) {
    for (auto& e : g->exec)
      if (e) (void)hipGraphExecDestroy(e), e = nullptr;
    g->key.clear();
  }
  if (cap) (void)hipStreamDestroy(cap), cap = nullptr;
}

void Hier::release_all() {
  for (hipEvent_t& e : pcg_ev)
    if (e) (void)hipEventDestroy(e), e = nullptr;
  if (pcg_status) (void)hipHostFree(pcg_status), pcg_status = nullptr;
  for (void* q : owned)
    if (p.release) p.release(q, p.alloc_ctx);
  owned.clear();
  for (void* q : owned_hip) (void)hipFree(q);
  owned_hip.clear();
}

// GMT_FORCE_L1_VARIANT=<cb> pins the level-1 sweep variant (0..3, 5..9, see the
// autotuner) for tests that compare every variant with the oracle.
static int forced_l1_variant() {
  const char* e = std::getenv("GMT_FORCE_L1_VARIANT");
  return e && *e ? std::atoi(e) : -1;
}

// GMT_FORCE_COARSE_VARIANT=<cb> pins the sweep variant of levels >= 2 (0..3:
// all cases or one case per thread, element- or neighbour-major) for tests.
static int forced_coarse_variant() {
  const char* e = std::getenv("GMT_FORCE_COARSE_VARIANT");
  return e && *e ? std::atoi(e) : -1;
}

template <typename T>
LevelView<T> Hier::view(int l) const {
  const LevelData& d = lv[l];
  LevelView<T> v{};
  v.N = d.N;
  v.n_n = d.n_n;
  v.node_lin = d.node_lin;
  v.node_map = d.node_map;
  v.elem_map = d.elem_map;
  v.occ8 = d.occ8;
  v.cmask = d.cmask;
  v.n_int = d.n_int;
  v.n_bnd = d.n_bnd;
  v.interior = d.interior;
  v.boundary = d.boundary;
  v.n_runs = d.n_runs;
  v.runs = d.runs;
  v.bnd_nbrs = d.bnd_nbrs;
  v.st_nodes = d.st_nodes;
  v.st_off = d.st_off;
  v.st_ids = d.st_ids;
  v.st_slot = d.st_slot;
  if constexpr (std::is_same<T, double>::value) {
    v.st_blk = d.st_blk64;
    v.n_st_blk = d.n_st_blk64;
    v.st_rest = d.st_rest64;
    v.n_st_rest = d.n_st_rest64;
  } else {
    v.st_blk = d.st_blk32;
    v.n_st_blk = d.n_st_blk32;
    v.st_rest = d.st_rest32;
    v.n_st_rest = d.n_st_rest32;
  }
  if constexpr (std::is_same<T, double>::value)
    v.oscale = d.oscale64;
  else
    v.oscale = d.oscale32;
  if constexpr (std::is_same<T, double>::value) {
    v.K = d.kind == KIND_SHARED ? Ke64 : (d.kind == KIND_TABLE ? table64 : d.Kel64);
    v.S = S64;
    v.kcls = kcls64;
    v.scls = scls64;
    v.bs = d.bs64;
    v.xcd = d.xcd64;
    v.cb = d.cb64;
  } else {
    v.K = d.kind == KIND_SHARED ? Ke32 : (d.kind == KIND_TABLE ? table32 : d.Kel32);
    v.S = S32;
    v.kcls = kcls32;
    v.scls = scls32;
    v.bs = d.bs32;
    v.xcd = d.xcd32;
    v.cb = d.cb32;
  }
  if (l > 0) {
    const int f = forced_coarse_variant();
    if (f >= 0 && f <= 3) v.cb = f;
  }
  if (l == 0) {
    const int f = forced_l1_variant();
    if (f >= 0 && f <= 9 && f != 4) v.cb = f;
    // a density hierarchy has only the scaled class-assembled boundary sweeps
    if (density && v.cb != 5 && v.cb != 7 && v.cb != 8) v.cb = 7;
    if (v.cb == 9 && v.n_st_blk == 0 && v.n_st_rest == 0) v.cb = 7;  // no staged tables
  }
  return v;
}

template <>
Work<float>& Hier::work<float>() {
  return w32;
}
template <>
Work<double>& Hier::work<double>() {
  return w64;
}

template <typename T>
void Hier::ensure_work() {
  Work<T>& W = work<T>();
  if (W.ready) return;
  W.f.assign(L, nullptr);
  W.u.assign(L, nullptr);
  W.io1.assign(L, nullptr);
  W.io2.assign(L, nullptr);
  W.io3.assign(L, nullptr);
  W.ualt.assign(L, nullptr);
  W.dvec.assign(L, nullptr);
  W.r.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    const size_t n = (size_t)lv[l].n_n * Q;
    if (l > 0) {
      W.f[l] = alloc<T>(n);
      W.u[l] = alloc<T>(n);
    }
    W.ualt[l] = alloc<T>(n);
    W.dvec[l] = alloc<T>(n);
    W.r[l] = alloc<T>(n);
  }
  const size_t n0 = (size_t)lv[0].n_n * Q;
  W.pr = alloc<T>(n0);
  W.pz = alloc<T>(n0);
  W.pp = alloc<T>(n0);
  W.pq = alloc<T>(n0);
  W.px = alloc<T>(n0);
  W.ready = true;
}

template <typename T>
void Hier::ensure_io(int l) {
  ensure_work<T>();
  Work<T>& W = work<T>();
  if (W.io1[l]) return;
  const size_t n = (size_t)lv[l].n_n * Q;
  W.io1[l] = alloc<T>(n);
  W.io2[l] = alloc<T>(n);
  W.io3[l] = alloc<T>(n);
}

template LevelView<float> Hier::view<float>(int) const;
template LevelView<double> Hier::view<double>(int) const;

// ================================================================ element constants (App. F)

// Trilinear shape-function gradients on the unit cube at point (px,py,pz);
// corner a = ax + 2 ay + 4 az.
static void shape_gradients(double px, double py, double pz, double g[8][3]) {
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const double fx = ax ? px : 1.0 - px, fy = ay ? py : 1.0 - py, fz = az ? pz : 1.0 - pz;
    const double sx = ax ? 1.0 : -1.0, sy = ay ? 1.0 : -1.0, sz = az ? 1.0 : -1.0;
    g[a][0] = sx * fy * fz;
    g[a][1] = fx * sy * fz;
    g[a][2] = fx * fy * sz;
  }
}

// K_e and X0 of the unit voxel (2x2x2 Gauss quadrature, exact for hex8),
// f_e = K_e X0 and C0 = X0^T K_e X0.
static void element_constants(Hier& h) {
  const int D = h.D, M = 8 * D, C = h.C;
  std::vector<double> K(M * M, 0.0), X(M * C, 0.0);
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  if (D == 3) {
    const double E = h.p.E, nu = h.p.nu;
    const double lam = E * nu / ((1 + nu) * (1 - 2 * nu)), G = E / (2 * (1 + nu));
    double Cm[6][6] = {{0}};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Cm[i][j] = lam + (i == j ? 2 * G : 0.0);
    Cm[3][3] = Cm[4][4] = Cm[5][5] = G;
    for (int qz = 0; qz < 2; ++qz)
      for (int qy = 0; qy < 2; ++qy)
        for (int qx = 0; qx < 2; ++qx) {
          double g[8][3];
          shape_gradients(gp[qx], gp[qy], gp[qz], g);
          // strain rows (11,22,33,23,13,12), engineering shear
          double B[6][24] = {{0}};
          for (int a = 0; a < 8; ++a) {
            B[0][3 * a + 0] = g[a][0];
            B[1][3 * a + 1] = g[a][1];
            B[2][3 * a + 2] = g[a][2];
            B[3][3 * a + 1] = g[a][2];
            B[3][3 * a + 2] = g[a][1];
            B[4][3 * a + 0] = g[a][2];
            B[4][3 * a + 2] = g[a][0];
            B[5][3 * a + 0] = g[a][1];
            B[5][3 * a + 1] = g[a][0];
          }
          double CB[6][24];
          for (int i = 0; i < 6; ++i)
            for (int j = 0; j < 24; ++j) {
              double s = 0;
              for (int k = 0; k < 6; ++k) s += Cm[i][k] * B[k][j];
              CB[i][j] = s;
            }
          for (int i = 0; i < 24; ++i)
            for (int j = 0; j < 24; ++j) {
              double s = 0;
              for (int k = 0; k < 6; ++k) s += B[k][i] * CB[k][j];
              K[i * M + j] += 0.125 * s;
            }
        }
    for (int a = 0; a < 8; ++a) {
      const double x = a & 1, y = (a >> 1) & 1, z = (a >> 2) & 1;
      X[(3 * a + 0) * C + 0] = x;
      X[(3 * a + 1) * C + 1] = y;
      X[(3 * a + 2) * C + 2] = z;
      X[(3 * a + 1) * C + 3] = 0.5 * z;
      X[(3 * a + 2) * C + 3] = 0.5 * y;
      X[(3 * a + 0) * C + 4] = 0.5 * z;
      X[(3 * a + 2) * C + 4] = 0.5 * x;
      X[(3 * a + 0) * C + 5] = 0.5 * y;
      X[(3 * a + 1) * C + 5] = 0.5 * x;
    }
  } else {
    for (int qz = 0; qz < 2; ++qz)
      for (int qy = 0; qy < 2; ++qy)
        for (int qx = 0; qx < 2; ++qx) {
          double g[8][3];
          shape_gradients(gp[qx], gp[qy], gp[qz], g);
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
              K[a * 8 + b] += 0.125 * h.p.kappa * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
        }
    for (int a = 0; a < 8; ++a) {
      X[a * C + 0] = a & 1;
      X[a * C + 1] = (a >> 1) & 1;
      X[a * C + 2] = (a >> 2) & 1;
    }
  }
  for (int i = 0; i < M * M; ++i) h.Ke[i] = K[i];
  for (int i = 0; i < M * C; ++i) h.X0[i] = X[i];
  for (int i = 0; i < M; ++i)
    for (int c = 0; c < C; ++c) {
      double s = 0;
      for (int j = 0; j < M; ++j) s += K[i * M + j] * X[j * C + c];
      h.fe[i * C + c] = s;
    }
  for (int c1 = 0; c1 < C; ++c1)
    for (int c2 = 0; c2 < C; ++c2) {
      double s = 0;
      for (int i = 0; i < M; ++i) s += X[i * C + c1] * h.fe[i * C + c2];
      h.C0[c1 * C + c2] = s;
    }
  double fn = 0;
  for (int i = 0; i < M * C; ++i) fn += h.fe[i] * h.fe[i];
  h.fe_norm = std::sqrt(fn);
}

// Ps[c][m][o]: weight of coarse-element corner o at corner m of child c
// (trilinear, App. E.1 restricted to one coarse cell).
static void local_prolongation(double Ps[8][8][8]) {
  for (int c = 0; c < 8; ++c)
    for (int m = 0; m < 8; ++m)
      for (int o = 0; o < 8; ++o) {
        double w = 1.0;
        for (int d = 0; d < 3; ++d) {
          const double pos = 0.5 * (((c >> d) & 1) + ((m >> d) & 1));
          w *= 1.0 - std::fabs(pos - ((o >> d) & 1));
        }
        Ps[c][m][o] = w;
      }
}

// 256-entry table of level-2 element matrices: entry mask = sum over children
// c in mask (ascending) of P_c^T K_e P_c.
static void mask_table(const Hier& h, const double Ps[8][8][8], std::vector<double>& tab) {
  const int D = h.D, M = 8 * D;
  std::vector<double> G(8 * M * M, 0.0);
  for (int c = 0; c < 8; ++c) {
    std::vector<double> T1(M * M, 0.0);
    for (int r = 0; r < M; ++r)
      for (int col = 0; col < M; ++col) {
        const int p = col / D, j = col % D;
        double s = 0;
        for (int n = 0; n < 8; ++n) s += h.Ke[r * M + n * D + j] * Ps[c][n][p];
        T1[r * M + col] = s;
      }
    for (int r = 0; r < M; ++r)
      for (int col = 0; col < M; ++col) {
        const int o = r / D, i = r % D;
        double s = 0;
        for (int m = 0; m < 8; ++m) s += Ps[c][m][o] * T1[(m * D + i) * M + col];
        G[(size_t)c * M * M + r * M + col] = s;
      }
  }
  tab.assign((size_t)256 * M * M, 0.0);
  for (int mask = 0; mask < 256; ++mask)
    for (int c = 0; c < 8; ++c)
      if (mask & (1 << c))
        for (int t = 0; t < M * M; ++t) tab[(size_t)mask * M * M + t] += G[(size_t)c * M * M + t];
}

// ================================================================ coarsest level

// Dense FP64 Cholesky of the pinned coarsest matrix and its explicit inverse.
// Auxiliary streams for independent setup work of one hierarchy (the power
// iterations of its levels), four per device, created on first use and kept
// for the life of the process; default priority, non-blocking.  Work on them
// is ordered against the caller's stream by events only, so hierarchies built
// at the same time from several threads may share them safely.
static hipStream_t aux_stream(int k) {
  static std::mutex mu;
  static std::map<int, std::vector<hipStream_t>> pool;
  int dev = 0;
  GMT_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  std::vector<hipStream_t>& v = pool[dev];
  if (v.empty()) {
    for (int i = 0; i < 4; ++i) {
      hipStream_t x = nullptr;
      GMT_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
      v.push_back(x);
    }
  }
  return v[(size_t)k % v.size()];
}

// Events (no timing) owned by a scope; destroyed when it ends.
struct EventSet {
  std::vector<hipEvent_t> ev;
  hipEvent_t make() {
    hipEvent_t e = nullptr;
    GMT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ev.push_back(e);
    return e;
  }
  ~EventSet() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
};

// The coarsest level's element matrices and connectivity on the host.
struct CoarseHost {
  std::vector<double> Ke;
  std::vector<int> en;
  double* dK = nullptr;
  int* dEN = nullptr;
  hipEvent_t ready = nullptr;
};

// Queues the copies of the coarsest level's element matrices and connectivity
// to the host on s; c.ready marks their completion.
static void coarse_fetch(Hier& h, hipStream_t s, CoarseHost& c, EventSet& evs) {
  const int l = h.L - 1;
  LevelData& d = h.lv[l];
  const int D = h.D, M = 8 * D;
  const int n = d.n_n * D;
  if (n > 2048) fail(GMT_E_INVAL, "coarsest level has %d DOFs (> 2048): use more levels", n);
  h.cn = n;
  c.dK = h.alloc<double>((size_t)d.n_e * M * M);
  c.dEN = h.alloc<int>((size_t)d.n_e * 8);
  launch_expand_elem_matrices(h.view<double>(l), d.kind, d.n_e, D, d.elem_lin, c.dK, s);
  launch_elem_nodes(d.elem_lin, d.n_e, d.node_map, d.N, c.dEN, s);
  c.Ke.resize((size_t)d.n_e * M * M);
  c.en.resize((size_t)d.n_e * 8);
  GMT_HIP(hipMemcpyAsync(c.Ke.data(), c.dK, c.Ke.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  GMT_HIP(hipMemcpyAsync(c.en.data(), c.dEN, c.en.size() * sizeof(int), hipMemcpyDeviceToHost, s));
  c.ready = evs.make();
  GMT_HIP(hipEventRecord(c.ready, s));
}

// Assembles, pins and inverts the coarsest operator on the host once the
// copies of coarse_fetch have landed (work queued on s after them keeps
// running meanwhile), then uploads the inverse on s and waits for s.
static void coarse_factor(Hier& h, hipStream_t s, CoarseHost& c) {
  const int l = h.L - 1;
  LevelData& d = h.lv[l];
  const int D = h.D, M = 8 * D;
  const int n = h.cn;
  GMT_HIP(hipEventSynchronize(c.ready));
  const std::vector<double>& Ke = c.Ke;
  const std::vector<int>& en = c.en;
  std::vector<double> A((size_t)n * n, 0.0);
  for (int e = 0; e < d.n_e; ++e)
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < D; ++i)
        for (int b = 0; b < 8; ++b)
          for (int j = 0; j < D; ++j)
            A[(size_t)(en[e * 8 + a] * D + i) * n + en[e * 8 + b] * D + j] +=
                Ke[(size_t)e * M * M + (a * D + i) * M + b * D + j];
  // pin node 0: identity rows / columns
  for (int i = 0; i < D; ++i) {
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = A[(size_t)j * n + i] = 0.0;
    A[(size_t)i * n + i] = 1.0;
  }
  double dmax = 0;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, A[(size_t)i * n + i]);
  // in-place lower Cholesky
  for (int j = 0; j < n; ++j) {
    double sjj = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) sjj -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(sjj > 1e-13 * dmax)) fail(GMT_E_SINGULAR, "coarsest Cholesky: pivot %d is %g", j, sjj);
    const double ljj = std::sqrt(sjj);
    A[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double sij = A[(size_t)i * n + j];
      const double* ri = &A[(size_t)i * n];
      const double* rj = &A[(size_t)j * n];
      for (int k = 0; k < j; ++k) sij -= ri[k] * rj[k];
      A[(size_t)i * n + j] = sij / ljj;
    }
  }
  // W = L^-1 (lower), then inv = W^T W
  std::vector<double> W((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    W[(size_t)c * n + c] = 1.0 / A[(size_t)c * n + c];
    for (int i = c + 1; i < n; ++i) {
      double sacc = 0;
      for (int k = c; k < i; ++k) sacc += A[(size_t)i * n + k] * W[(size_t)k * n + c];
      W[(size_t)i * n + c] = -sacc / A[(size_t)i * n + i];
    }
  }
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double sacc = 0;
      for (int k = i; k < n; ++k) sacc += W[(size_t)k * n + i] * W[(size_t)k * n + j];
      inv[(size_t)i * n + j] = inv[(size_t)j * n + i] = sacc;
    }
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < n; ++j) inv[(size_t)i * n + j] = inv[(size_t)j * n + i] = 0.0;
  h.cinv64 = h.alloc<double>((size_t)n * n);
  h.cinv32 = h.alloc<float>((size_t)n * n);
  GMT_HIP(hipMemcpyAsync(h.cinv64, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, s));
  launch_convert<double, float>(h.cinv64, h.cinv32, inv.size(), s);
  GMT_HIP(hipStreamSynchronize(s));
  h.release(c.dK);
  h.release(c.dEN);
}

// ================================================================ building blocks

template <typename T>
static const T* dinv_of(const Hier& h, int l) {
  if constexpr (std::is_same<T, double>::value)
    return h.lv[l].dinv64;
  else
    return h.lv[l].dinv32;
}

template <typename T>
static void apply(Hier& h, int l, int epi, const T* u, const T* f, T* out, int C, hipStream_t s,
                  T omega = 0, T rho1 = 0, T rho2 = 0, T* dvec = nullptr, const LevelView<T>* view = nullptr,
                  const T* dvec_in = nullptr) {
  EpiArgs<T> e{};
  e.f = f;
  e.dinv = dinv_of<T>(h, l);
  e.dvec = dvec;
  e.dvec_in = dvec_in ? dvec_in : dvec;
  e.out = out;
  e.omega = omega;
  e.rho1 = rho1;
  e.rho2 = rho2;
  launch_apply<T>(view ? *view : h.view<T>(l), h.lv[l].kind, h.D, C, epi, u, e, s);
}

struct CycleCfg {
  int nu1 = 2, nu2 = 2, smoother = GMT_SMOOTH_CHEBYSHEV, schedule = GMT_CYCLE_V;
  std::vector<double> omega, lo, hi;
};

// ------------------------------------------------------------ colour classes (Gauss-Seidel)
// Node ids of every level split by colour x mod 2 + 2 (y mod 2) + 4 (z mod 2)
// (stable: ascending id inside a colour); level 1 splits its interior and
// boundary lists the same way and rebuilds the boundary neighbour table in the
// order of the split list.  Built once per hierarchy, on the calling thread.
static void split_by_colour(const std::vector<int>& ids, const std::vector<int>& lin, int N, std::vector<int>& out,
                            int off[9]) {
  int cnt[8] = {0};
  auto colour = [&](int i) {
    const int v = lin[i];
    return (v % N) % 2 + 2 * (((v / N) % N) % 2) + 4 * ((v / (N * N)) % 2);
  };
  for (int i : ids) ++cnt[colour(i)];
  off[0] = 0;
  for (int c = 0; c < 8; ++c) off[c + 1] = off[c] + cnt[c];
  out.assign(ids.size(), 0);
  int pos[8];
  for (int c = 0; c < 8; ++c) pos[c] = off[c];
  for (int i : ids) out[pos[colour(i)]++] = i;
}

static void ensure_colours(Hier& h, hipStream_t s) {
  for (int l = 0; l + 1 < h.L; ++l) {
    LevelData& d = h.lv[l];
    if (d.col_nodes) continue;
    std::vector<int> lin(d.n_n), ids(d.n_n), out;
    GMT_HIP(hipMemcpyAsync(lin.data(), d.node_lin, d.n_n * sizeof(int), hipMemcpyDeviceToHost, s));
    GMT_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < d.n_n; ++i) ids[i] = i;
    split_by_colour(ids, lin, d.N, out, d.col_off);
    d.col_nodes = h.alloc<int>(d.n_n);
    GMT_HIP(hipMemcpyAsync(d.col_nodes, out.data(), d.n_n * sizeof(int), hipMemcpyHostToDevice, s));
    GMT_HIP(hipStreamSynchronize(s));
    if (l > 0) continue;
    for (int part = 0; part < 2; ++part) {
      const int cnt = part == 0 ? d.n_int : d.n_bnd;
      const int* src = part == 0 ? d.interior : d.boundary;
      int* off = part == 0 ? d.col_int_off : d.col_bnd_off;
      for (int c = 0; c < 9; ++c) off[c] = 0;
      if (cnt == 0) continue;
      ids.resize(cnt);
      GMT_HIP(hipMemcpyAsync(ids.data(), src, cnt * sizeof(int), hipMemcpyDeviceToHost, s));
      GMT_HIP(hipStreamSynchronize(s));
      split_by_colour(ids, lin, d.N, out, off);
      int* dst = h.alloc<int>(cnt);
      GMT_HIP(hipMemcpyAsync(dst, out.data(), cnt * sizeof(int), hipMemcpyHostToDevice, s));
      GMT_HIP(hipStreamSynchronize(s));
      if (part == 0) {
        d.col_int = dst;
      } else {
        d.col_bnd = dst;
        d.col_bnd_nbrs = h.alloc<int>((size_t)cnt * kBndStride);
        if (reinterpret_cast<uintptr_t>(d.col_bnd_nbrs) % 16 != 0)
          fail(GMT_E_STATE, "boundary neighbour table is not 16-byte aligned");
        launch_boundary_nbrs(d.col_bnd, cnt, d.node_lin, d.node_map, d.N, d.col_bnd_nbrs, s);
        GMT_HIP(hipStreamSynchronize(s));
      }
    }
  }
}

// The operator sweep of level l restricted to the nodes of colour c.
template <typename T>
static LevelView<T> colour_view(const Hier& h, int l, int c) {
  const LevelData& d = h.lv[l];
  LevelView<T> v = h.view<T>(l);
  if (l == 0) {
    v.interior = d.col_int ? d.col_int + d.col_int_off[c] : nullptr;
    v.n_int = d.col_int_off[c + 1] - d.col_int_off[c];
    v.boundary = d.col_bnd ? d.col_bnd + d.col_bnd_off[c] : nullptr;
    v.n_bnd = d.col_bnd_off[c + 1] - d.col_bnd_off[c];
    v.bnd_nbrs = d.col_bnd_nbrs ? d.col_bnd_nbrs + (size_t)d.col_bnd_off[c] * kBndStride : nullptr;
    v.n_runs = 0;
    v.runs = nullptr;
    if (v.cb < 5 || v.cb > 8) v.cb = 7;  // the list-driven variants
  } else {
    v.list = d.col_nodes + d.col_off[c];
    v.n_list = d.col_off[c + 1] - d.col_off[c];
  }
  return v;
}

static CycleCfg make_cycle(const Hier& h, const gmt_cycle_opts* o) {
  CycleCfg c;
  if (o) {
    c.nu1 = o->nu1;
    c.nu2 = o->nu2;
    if (c.nu1 == 0 && c.nu2 == 0) c.nu1 = c.nu2 = 2;
    c.smoother = o->smoother;
    c.schedule = o->schedule;
  }
  if (c.nu1 < 0 || c.nu2 < 0 || c.nu1 > 64 || c.nu2 > 64) fail(GMT_E_INVAL, "smoothing degree out of range");
  if (c.smoother != GMT_SMOOTH_CHEBYSHEV && c.smoother != GMT_SMOOTH_JACOBI && c.smoother != GMT_SMOOTH_GS)
    fail(GMT_E_INVAL, "bad smoother");
  if (c.schedule != GMT_CYCLE_V && c.schedule != GMT_CYCLE_W && c.schedule != GMT_CYCLE_F)
    fail(GMT_E_INVAL, "bad cycle schedule");
  for (int l = 0; l < h.L; ++l) {
    const double lam = h.lv[l].lam;
    const double w0 = c.smoother == GMT_SMOOTH_GS ? 1.0 : 4.0 / (3.0 * lam);
    c.omega.push_back(o && o->omega ? o->omega[l] : w0);
    if (c.smoother == GMT_SMOOTH_GS && !(c.omega[l] > 0 && c.omega[l] < 2))
      fail(GMT_E_INVAL, "Gauss-Seidel / SOR weight of level %d outside (0, 2)", l + 1);
    c.lo.push_back(o && o->lo ? o->lo[l] : lam / 30.0);
    c.hi.push_back(o && o->hi ? o->hi[l] : 1.1 * lam);
    if (c.smoother == GMT_SMOOTH_CHEBYSHEV && !(c.hi[l] > c.lo[l] && c.lo[l] > 0))
      fail(GMT_E_INVAL, "Chebyshev interval of level %d is not 0 < lo < hi", l + 1);
  }
  return c;
}

// nu smoothing steps on level l; u / ualt are swapped so that u holds the result.
// Gauss-Seidel (p1 = omega) runs the colours 0..7, or 7..0 when `post` (the
// adjoint order, for the post-smoother), each colour as the residual at its
// nodes followed by the in-place update there.
template <typename T>
static void smooth(Hier& h, int l, const T* f, T*& u, T*& ualt, T* dvec, int nu, bool zero_start,
                   int smoother, double p1, double p2, hipStream_t s, bool post = false) {
  const int n = h.lv[l].n_n;
  if (nu <= 0) {
    if (zero_start) launch_fill<T>(u, (size_t)n * h.Q, T(0), s);
    return;
  }
  const T* dinv = dinv_of<T>(h, l);
  if (smoother == GMT_SMOOTH_GS) {
    const LevelData& d = h.lv[l];
    if (!d.col_nodes) fail(GMT_E_STATE, "colour classes of level %d are not built", l + 1);
    if (zero_start) launch_fill<T>(u, (size_t)n * h.Q, T(0), s);
    T* r = h.work<T>().r[l];
    for (int it = 0; it < nu; ++it)
      for (int k = 0; k < 8; ++k) {
        const int c = post ? 7 - k : k;
        const int cnt = d.col_off[c + 1] - d.col_off[c];
        if (cnt == 0) continue;
        const LevelView<T> v = colour_view<T>(h, l, c);
        apply<T>(h, l, EPI_RESID, u, f, r, h.C, s, T(0), T(0), T(0), nullptr, &v);
        launch_gs_update<T>(d.col_nodes + d.col_off[c], cnt, n, h.D, h.C, dinv, r, u, (T)p1, s);
      }
    return;
  }
  if (smoother == GMT_SMOOTH_JACOBI) {
    const T omega = (T)p1;
    for (int it = 0; it < nu; ++it) {
      if (it == 0 && zero_start) {
        launch_smooth_zero<T>(n, h.D, h.C, f, dinv, omega, u, nullptr, s);
      } else {
        apply<T>(h, l, EPI_JACOBI, u, f, ualt, h.C, s, omega);
        std::swap(u, ualt);
      }
    }
    return;
  }
  const double lo = p1, hi = p2;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho = 1.0 / sigma;
  // A first step from zero leaves the direction equal to the iterate
  // (d = u = D^-1 f / theta): it writes u only, and the next step reads the
  // direction from u (one pass over a vector saved).  With a single step the
  // direction is written too, for whoever reads it after the smoother.
  bool d_in_u = false;
  if (zero_start) {
    d_in_u = nu > 1;
    launch_smooth_zero<T>(n, h.D, h.C, f, dinv, (T)(1.0 / theta), u, d_in_u ? nullptr : dvec, s);
  } else {
    apply<T>(h, l, EPI_CHEB0, u, f, ualt, h.C, s, T(0), T(0), (T)(1.0 / theta), dvec);
    std::swap(u, ualt);
  }
  for (int k = 1; k < nu; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    apply<T>(h, l, EPI_CHEB, u, f, ualt, h.C, s, T(0), (T)(rn * rho), (T)(2.0 * rn / delta), dvec, nullptr,
             d_in_u ? u : nullptr);
    d_in_u = false;
    std::swap(u, ualt);
    rho = rn;
  }
}

template <typename T>
static const T* cinv_of(const Hier& h) {
  if constexpr (std::is_same<T, double>::value)
    return h.cinv64;
  else
    return h.cinv32;
}

// Iterates and right-hand sides of the levels during one cycle.
template <typename T>
struct CycleState {
  std::vector<T*> cur, alt;
  std::vector<const T*> f;
  std::vector<char> entered;
  const T* const* e_init;
};

// One visit of level l (Alg. 1 / Alg. 2 recursion): pre-smoothing, residual,
// restriction, the coarse correction problem treated by the schedule (one
// visit of level l+1 for V, two in a row for W, an F-visit then a V-visit for
// F; the exact coarsest solve is never repeated: a second one changes
// nothing), prolongation and post-smoothing.  Level l+1 starts from zero, or
// from its injected correction e_hat^{l+1} at its first entry in the cycle.
template <typename T>
static void cycle_visit(Hier& h, int l, bool zero_start, int sched, CycleState<T>& st, const CycleCfg& cfg,
                        hipStream_t s) {
  Work<T>& W = h.work<T>();
  const int L = h.L;
  if (l == L - 1) {
    launch_coarse_solve<T>(cinv_of<T>(h), h.cn, h.D, h.C, st.f[l], st.cur[l], s);
    return;
  }
  const double p1 = cfg.smoother == GMT_SMOOTH_CHEBYSHEV ? cfg.lo[l] : cfg.omega[l];
  const double p2 = cfg.hi[l];
  smooth<T>(h, l, st.f[l], st.cur[l], st.alt[l], W.dvec[l], cfg.nu1, zero_start, cfg.smoother, p1, p2, s);
  apply<T>(h, l, EPI_RESID, st.cur[l], st.f[l], W.r[l], h.C, s);
  const int c = l + 1;
  launch_restrict<T>(h.view<T>(l), h.view<T>(c), h.Q, h.D, W.r[l], W.f[c], s);
  st.f[c] = W.f[c];
  st.cur[c] = W.u[c];
  st.alt[c] = W.ualt[c];
  bool zs = true;
  if (st.e_init && st.e_init[c] && c < L - 1 && !st.entered[c]) {
    launch_copy<T>(st.e_init[c], st.cur[c], (size_t)h.lv[c].n_n * h.Q, s);
    zs = false;
  }
  st.entered[c] = 1;
  if (sched == GMT_CYCLE_V) {
    cycle_visit<T>(h, c, zs, GMT_CYCLE_V, st, cfg, s);
  } else if (sched == GMT_CYCLE_W) {
    cycle_visit<T>(h, c, zs, GMT_CYCLE_W, st, cfg, s);
    if (c < L - 1) cycle_visit<T>(h, c, false, GMT_CYCLE_W, st, cfg, s);
  } else {
    cycle_visit<T>(h, c, zs, GMT_CYCLE_F, st, cfg, s);
    if (c < L - 1) cycle_visit<T>(h, c, false, GMT_CYCLE_V, st, cfg, s);
  }
  launch_prolong_add<T>(h.view<T>(l), h.view<T>(c), h.Q, h.D, st.cur[c], st.cur[l], s);
  smooth<T>(h, l, st.f[l], st.cur[l], st.alt[l], W.dvec[l], cfg.nu2, false, cfg.smoother, p1, p2, s, true);
}

// One multigrid cycle (Alg. 2; the schedule of cfg) in precision T on caller
// buffers f0 / u0 of level l0 (the finest level for the solver; l0 > 0 runs the
// sub-cycle of the coarser levels, used by the adjoint of the learned path).
template <typename T>
static void vcycle(Hier& h, const T* f0, T* u0, bool u0_zero, const T* const* e_init, const CycleCfg& cfg,
                   hipStream_t s, int l0 = 0, const T** result = nullptr) {
  h.ensure_work<T>();
  Work<T>& W = h.work<T>();
  const int L = h.L;
  CycleState<T> st;
  st.cur.assign(L, nullptr);
  st.alt.assign(L, nullptr);
  st.f.assign(L, nullptr);
  st.entered.assign(L, 0);
  st.e_init = e_init;
  st.cur[l0] = u0;
  st.alt[l0] = W.ualt[l0];
  st.f[l0] = f0;
  cycle_visit<T>(h, l0, u0_zero, cfg.schedule, st, cfg, s);
  // the smoothers ping-pong between u0 and a work buffer; a caller that passes
  // `result` takes the iterate where it ended (the same buffer for the same
  // cycle configuration) instead of a copy back into u0
  if (result)
    *result = st.cur[l0];
  else if (st.cur[l0] != u0)
    launch_copy<T>(st.cur[l0], u0, (size_t)h.lv[l0].n_n * h.Q, s);
}

// ------------------------------------------------------------ launch-shape autotuner
// The operator sweeps of a level have a launch shape: workgroup size (256 or
// 64), cases per thread (all c, or 1 with one grid row per case) and plain or
// XCD-contiguous workgroup numbering; level 1 always uses 256-wide groups and
// chooses between one pass over the neighbourhood for all cases (boundary
// nodes as a masked stencil, cb 0, or element by element, cb 2) and one pass
// per case (cb 1, or cb 3 with interior nodes in runs along x), or takes the
// boundary nodes as a masked stencil assembled in registers from the symmetry
// classes of K_e, with the interior one case per pass (cb 5; cb 7 with all 27
// neighbours of a case loaded before the arithmetic; cb 9 with the distinct
// neighbours of each group of 256 or 512 interior nodes staged in LDS) or all
// cases per neighbour load (cb 6).
// Before the first solve of a hierarchy, every
// candidate is timed on every level (K.u on the work vectors: 2 warm-up and 3
// timed launches between HIP events) and the fastest is kept.  Choices are
// cached per (d, c, precision, operator kind, log2 of the node count, node
// density class), so later hierarchies of the same class reuse them without
// timing.  GMT_AUTOTUNE=0 keeps the defaults (256 wide, all cases, XCD order).
struct Shape {
  int bs, cb, xcd;
};
static std::mutex g_tune_mu;
static std::map<std::vector<int>, Shape> g_tune;

template <typename T>
static void autotune(Hier& h, hipStream_t s) {
  const bool f32 = !std::is_same<T, double>::value;
  const char* env = std::getenv("GMT_AUTOTUNE");
  const bool off = env && std::string(env) == "0";
  h.ensure_work<T>();
  Work<T>& W = h.work<T>();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  for (int l = 0; l < h.L; ++l) {
    LevelData& d = h.lv[l];
    bool& tuned = f32 ? d.tuned32 : d.tuned64;
    int& bs = f32 ? d.bs32 : d.bs64;
    int& xcd = f32 ? d.xcd32 : d.xcd64;
    int& cb = f32 ? d.cb32 : d.cb64;
    if (tuned) continue;
    tuned = true;
    if (off || d.n_n == 0) continue;
    int nb = 0;
    while ((1 << (nb + 1)) <= d.n_n) ++nb;
    const double dens = (double)d.n_n / ((double)d.N * d.N * d.N);
    const std::vector<int> key = {h.D, h.C, f32 ? 32 : 64, d.kind, nb, (int)(dens * 8.0), h.density ? 1 : 0};
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        bs = it->second.bs;
        cb = it->second.cb;
        xcd = it->second.xcd;
        continue;
      }
    }
    if (!e0) {
      GMT_HIP(hipEventCreate(&e0));
      GMT_HIP(hipEventCreate(&e1));
    }
    T* x = l == 0 ? W.pr : W.u[l];
    T* y = l == 0 ? W.pz : W.r[l];
    launch_fill<T>(x, (size_t)d.n_n * h.Q, T(0), s);
    // level 1: the variants that have won on some cell shape (the others stay
    // selectable through GMT_FORCE_L1_VARIANT)
    std::vector<Shape> cand = {{256, 0, 1}, {256, 0, 0}};
    if (l == 0 && h.density) {
      cand = {{256, 7, 1}, {256, 7, 0}, {256, 5, 1}, {256, 8, 1}, {256, 8, 0}};
    } else if (l == 0) {
      cand = {{256, 8, 1}, {256, 8, 0}, {256, 7, 1}, {256, 7, 0}, {256, 5, 1}, {256, 6, 1}, {256, 6, 0}};
      if ((f32 ? d.n_st_blk32 : d.n_st_blk64) > 0) cand.insert(cand.end(), {{256, 9, 1}, {256, 9, 0}});
      if (h.C > 1) cand.insert(cand.end(), {{256, 1, 1}, {256, 1, 0}});
    }
    if (l > 0) {
      cand.insert(cand.end(), {{64, 0, 1}, {64, 0, 0}, {64, 2, 1}, {64, 2, 0}});
      if (h.C > 1) cand.insert(cand.end(), {{256, 1, 1}, {256, 1, 0}, {64, 1, 1}, {64, 1, 0}, {64, 3, 1}});
    }
    float best = INFINITY;
    Shape pick = cand[0];
    for (const Shape& c : cand) {
      bs = c.bs;
      cb = c.cb;
      xcd = c.xcd;
      for (int r = 0; r < 5; ++r) {
        if (r == 2) GMT_HIP(hipEventRecord(e0, s));
        apply<T>(h, l, EPI_KU, x, nullptr, y, h.C, s);
      }
      GMT_HIP(hipEventRecord(e1, s));
      GMT_HIP(hipEventSynchronize(e1));
      float ms = 0;
      GMT_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (std::getenv("GMT_TIMING"))
        fprintf(stderr, "[gmt tune]   level %d candidate bs %d cb %d xcd %d: %.1f us\n", l + 1, c.bs, c.cb, c.xcd,
                ms * 1e3 / 3);
      if (ms < best) {
        best = ms;
        pick = c;
      }
    }
    bs = pick.bs;
    cb = pick.cb;
    xcd = pick.xcd;
    if (std::getenv("GMT_TIMING"))
      fprintf(stderr, "[gmt tune] level %d (%s, n_n %d): bs %d cb %d xcd %d, %.1f us\n", l + 1,
              f32 ? "f32" : "f64", d.n_n, bs, cb, xcd, best * 1e3 / 3);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = pick;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
}

static void host_dot(Hier& h, const double* dev, int n, double* out, hipStream_t s) {
  GMT_HIP(hipMemcpyAsync(out, dev, n * sizeof(double), hipMemcpyDeviceToHost, s));
  GMT_HIP(hipStreamSynchronize(s));
}

// Inner PCG on K x = b from x = 0, V-cycle preconditioned.  The periodic
// system is singular (rigid translations, constant per DOF component, span the
// null space) and consistent in exact arithmetic.  Rounding re-introduces a
// translation component into r every iteration; the pinned coarsest solve would
// turn it into a large spurious correction, so CG runs on the range of K: the
// preconditioner is M^-1 = Pi V Pi with Pi the projection that removes the
// column means (symmetric, so CG stays valid).
// Stops when ||r_m|| <= tol[m] * ||b_m|| for every case, after maxit
// iterations, or when the residual stagnates.
// Records body() on the hierarchy's capture stream as an executable graph.
template <typename F>
static hipGraphExec_t capture_graph(Hier& h, F&& body) {
  if (!h.cap) GMT_HIP(hipStreamCreateWithFlags(&h.cap, hipStreamNonBlocking));
  GMT_HIP(hipStreamBeginCapture(h.cap, hipStreamCaptureModeThreadLocal));
  try {
    body(h.cap);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(h.cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipGraph_t g = nullptr;
  GMT_HIP(hipStreamEndCapture(h.cap, &g));
  hipGraphExec_t e = nullptr;
  const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (err != hipSuccess) fail(GMT_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(err));
  return e;
}

template <typename T>
static Hier::PcgGraphs& graphs_of(Hier& h) {
  if constexpr (std::is_same<T, double>::value)
    return h.g64;
  else
    return h.g32;
}

// inner PCG gives up after this many iterations without a 2 % gain in the
// worst case's residual ratio (ill-conditioned cells plateau for a while
// before converging, so the window is generous)
constexpr int kStagnation = 300;

// MIXED (T = double only): the Krylov vectors, dot products and the K.p
// product stay FP64, and only the preconditioner runs in FP32 — the residual
// is rounded to FP32, one FP32 V-cycle is applied and its result widened
// again.  The CG recurrence then keeps FP64 accuracy (its iteration count
// is the FP64 one) at close to the FP32 cost of a V-cycle.
template <typename T, bool MIXED = false>
static int pcg(Hier& h, const T* b, T* x, const double* tol, int maxit, int check_every, bool graph,
               const CycleCfg& cfg, hipStream_t s, bool* reached = nullptr) {
  static_assert(!MIXED || std::is_same<T, double>::value, "the mixed PCG keeps FP64 Krylov vectors");
  if (reached) *reached = false;
  h.ensure_work<T>();
  if (MIXED) h.ensure_work<float>();
  Work<T>& W = h.work<T>();
  Work<float>& W32 = h.work<float>();
  const int n = h.lv[0].n_n, C = h.C, D = h.D, Q = h.Q;
  const size_t tot = (size_t)n * Q;
  double* sc = h.red_out;
  double *rz = sc, *pq = sc + 8, *alpha = sc + 16, *beta = sc + 24, *rzn = sc + 32, *rr = sc + 40;
  double* sums = sc + 200;
  double* sums_z = sc + 224;  // column sums of the preconditioned residual
  double* sums_q = sc + 100;  // column sums of K p
  const double inv_n = n > 0 ? 1.0 / n : 0.0;
  double bn2[8], rr_h[8];
  launch_fill<T>(x, tot, T(0), s);
  launch_copy<T>(b, W.pr, tot, s);
  launch_project<T>(W.pr, n, Q, D, h.red_partial, sums, s);
  launch_dot<T>(W.pr, W.pr, n, C, D, h.red_partial, rr, s);
  host_dot(h, rr, C, bn2, s);
  // z = Pi V(r): the V-cycle in T, or (MIXED) in FP32 on the rounded residual; z is
  // left where the cycle ends (W.pz or the level's work buffer, fixed for the cycle
  // configuration) and its projection Pi is applied on the fly by the consumers:
  // the column sums, then the dot r.z and the direction update read z minus its
  // means (bit for bit what projecting z in place gives)
  const T* z = W.pz;
  auto vc = [&](hipStream_t st) {
    if constexpr (MIXED) {
      launch_convert<double, float>(W.pr, W32.pr, tot, st);
      const float* z32 = W32.pz;
      vcycle<float>(h, W32.pr, W32.pz, true, nullptr, cfg, st, 0, &z32);
      launch_convert<float, double>(z32, W.pz, tot, st);
      z = W.pz;
    } else {
      vcycle<T>(h, W.pr, W.pz, true, nullptr, cfg, st, 0, &z);
    }
  };
  // rzn = r . Pi z and p = Pi z + beta p
  auto finish_direction = [&](hipStream_t st, const double* fl) {
    launch_colsum<T>(z, n, Q, D, h.red_partial, sums_z, st);
    launch_dot_centered<T>(W.pr, z, sums_z, inv_n, n, C, D, h.red_partial, rzn, st);
    launch_pcg_beta(rzn, rz, beta, C, st, fl);
    launch_pcg_direction<T>(W.pp, z, beta, n, Q, D, st, sums_z, inv_n);
  };
  vc(s);
  launch_colsum<T>(z, n, Q, D, h.red_partial, sums_z, s);
  launch_dot_centered<T>(W.pr, z, sums_z, inv_n, n, C, D, h.red_partial, rz, s);
  launch_fill<T>(W.pp, tot, T(0), s);
  launch_fill<double>(beta, C, 0.0, s);
  launch_pcg_direction<T>(W.pp, z, beta, n, Q, D, s, sums_z, inv_n);  // p = Pi z
  int it = 0;
  double best = INFINITY;
  int since_best = 0;
  // convergence test on the host copy rr_h: returns true when every case is done;
  // tracks the progress measure max_m ||r_m|| / (tol_m ||b_m||) for stagnation
  double worst = INFINITY;
  auto converged = [&]() {
    bool done = true;
    worst = 0;
    for (int c = 0; c < C; ++c) {
      if (!std::isfinite(rr_h[c])) fail(GMT_E_NOCONV, "PCG residual of case %d is not finite", c);
      const double target = tol[c] * std::sqrt(bn2[c]);
      if (std::sqrt(rr_h[c]) > target) done = false;
      if (target > 0) worst = std::max(worst, std::sqrt(rr_h[c]) / target);
    }
    return done;
  };
  if (graph) {
    // Device-side convergence: flags [0] stop, [1] iterations run, [2 + m] the
    // squared target of case m.  Every captured iteration ends with ||r_m||^2 and
    // k_pcg_check, which sets the stop flag once every case meets its target;
    // from then on alpha = beta = 0, so the rest of a block (and a block
    // launched ahead) leaves x and r unchanged.
    if (!h.pcg_flags) h.pcg_flags = h.alloc<double>(16);
    if (!h.pcg_status) GMT_HIP(hipHostMalloc((void**)&h.pcg_status, 2 * 16 * sizeof(double), hipHostMallocDefault));
    for (hipEvent_t& e : h.pcg_ev)
      if (!e) GMT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    double* fl = h.pcg_flags;
    {
      double init[16] = {0};
      for (int c = 0; c < C; ++c) {
        const double t = tol[c] * std::sqrt(bn2[c]);
        init[2 + c] = t * t;
      }
      GMT_HIP(hipMemcpyAsync(fl, init, sizeof(init), hipMemcpyHostToDevice, s));
      GMT_HIP(hipStreamSynchronize(s));
    }
    // one iteration after the initial preconditioning, as in the launch-by-launch
    // loop below, ending with the residual norms and the convergence check
    // The residual is kept free of rigid translations by removing the column
    // means of q = K p in the update (K p has none in exact arithmetic; the sums
    // come with p.q in one pass), instead of projecting r after it; r.z and r.r
    // share one pass over r.
    auto step = [&](hipStream_t st) {
      apply<T>(h, 0, EPI_KU, W.pp, nullptr, W.pq, C, st);
      launch_dot_colsum<T>(W.pp, W.pq, n, C, D, h.red_partial, pq, sums_q, st);
      launch_pcg_alpha(rz, pq, alpha, C, st, fl);
      launch_pcg_update<T>(x, W.pr, W.pp, W.pq, alpha, n, Q, D, st, sums_q, inv_n);
      vc(st);
      launch_colsum<T>(z, n, Q, D, h.red_partial, sums_z, st);
      launch_dot2_centered<T>(W.pr, z, sums_z, inv_n, n, C, D, h.red_partial, rzn, rr, st);
      launch_pcg_beta(rzn, rz, beta, C, st, fl);
      launch_pcg_direction<T>(W.pp, z, beta, n, Q, D, st, sums_z, inv_n);
      launch_pcg_check(rr, C, fl, st);
    };
    Hier::PcgGraphs& G = MIXED ? h.gmx : graphs_of<T>(h);
    std::vector<double> key = {(double)(uintptr_t)x, (double)cfg.nu1, (double)cfg.nu2, (double)cfg.smoother,
                               (double)cfg.schedule};
    for (int l = 0; l < h.L; ++l) key.insert(key.end(), {cfg.omega[l], cfg.lo[l], cfg.hi[l]});
    if (G.key != key) {
      for (auto& e : G.exec)
        if (e) (void)hipGraphExecDestroy(e), e = nullptr;
      G.key.clear();
      const int steps[2] = {1, 4};
      for (int k = 0; k < 2; ++k)
        G.exec[k] = capture_graph(h, [&](hipStream_t st) {
          for (int i = 0; i < steps[k]; ++i) step(st);
        });
      G.key = key;
    }
    // progress measure before the first iteration: ||r_m|| = ||b_m||
    worst = 0;
    for (int c = 0; c < C; ++c)
      if (bn2[c] > 0 && tol[c] > 0) worst = std::max(worst, 1.0 / tol[c]);
    double prev = -1;
    int prev_k = 1;
    // Blocks of 1 or 4 iterations, each followed by an asynchronous copy of the
    // flags and ||r_m||^2 into a pinned slot and an event.  While the observed
    // convergence rate predicts more than four iterations beyond those already
    // in flight, a second block is queued before the host waits for the first,
    // so the GPU does not idle on the host round trip.
    struct Pending {
      int slot, k;
    };
    Pending q[2];
    int nq = 0, launched = 0, inflight = 0, next_slot = 0;
    auto remaining = [&]() -> double {  // predicted iterations to the target from the last observation
      if (!(prev > 0 && worst < prev && std::isfinite(worst))) return 0.0;
      const double rate = std::pow(worst / prev, 1.0 / prev_k);
      if (!(rate < 1)) return 0.0;
      return std::log(worst) / -std::log(rate);
    };
    auto launch_block = [&](int k) {
      double* slot = h.pcg_status + 16 * next_slot;
      GMT_HIP(hipGraphLaunch(G.exec[k == 1 ? 0 : 1], s));
      GMT_HIP(hipMemcpyAsync(slot, fl, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
      GMT_HIP(hipMemcpyAsync(slot + 2, rr, C * sizeof(double), hipMemcpyDeviceToHost, s));
      GMT_HIP(hipEventRecord(h.pcg_ev[next_slot], s));
      q[nq++] = {next_slot, k};
      next_slot ^= 1;
      launched += k;
      inflight += k;
    };
    auto observe = [&]() -> bool {  // oldest block: true when its flag says stop
      const Pending pb = q[0];
      q[0] = q[1];
      --nq;
      GMT_HIP(hipEventSynchronize(h.pcg_ev[pb.slot]));
      const double* slot = h.pcg_status + 16 * pb.slot;
      it = (int)slot[1];
      for (int c = 0; c < C; ++c) rr_h[c] = slot[2 + c];
      inflight -= pb.k;
      prev = worst;
      prev_k = pb.k;
      return slot[0] != 0.0;
    };
    try {
      while (true) {
        while (launched < maxit && nq < 2) {
          const double rem = remaining() - inflight;
          const int k = (rem > 4.0 && maxit - launched >= 4) ? 4 : 1;
          if (nq > 0 && k == 1) break;  // near the target: one block at a time
          launch_block(k);
          if (k == 1) break;
        }
        if (nq == 0) break;  // maxit launched and observed
        const bool stop = observe();
        const bool done = converged();  // (fails on a non-finite residual)
        if (stop || done) {
          if (reached) *reached = true;
          break;
        }
        if (worst < 0.98 * best) {
          best = worst;
          since_best = 0;
        } else if ((since_best += prev_k) >= kStagnation) {
          break;  // stagnation: hand back to the FP64 refinement loop
        }
      }
    } catch (...) {
      (void)hipStreamSynchronize(s);
      throw;
    }
    // a block still in flight is gated once the flag is set; after a stagnation
    // stop it runs on as ordinary iterations: wait for it and take its count
    while (nq > 0) observe();
    return it;
  }
  while (it < maxit) {
    ++it;
    apply<T>(h, 0, EPI_KU, W.pp, nullptr, W.pq, C, s);
    launch_dot_colsum<T>(W.pp, W.pq, n, C, D, h.red_partial, pq, sums_q, s);
    launch_pcg_alpha(rz, pq, alpha, C, s);
    launch_pcg_update<T>(x, W.pr, W.pp, W.pq, alpha, n, Q, D, s, sums_q, inv_n);
    if (it % check_every == 0 || it == maxit) {
      launch_dot<T>(W.pr, W.pr, n, C, D, h.red_partial, rr, s);
      host_dot(h, rr, C, rr_h, s);
      if (converged()) {
        if (reached) *reached = true;
        break;
      }
      if (worst < 0.98 * best) {
        best = worst;
        since_best = 0;
      } else if ((since_best += check_every) >= kStagnation) {
        break;  // stagnation: hand back to the FP64 refinement loop
      }
    }
    vc(s);
    finish_direction(s, nullptr);
  }
  return it;
}

// FP64 relative residual per case of u64 against f64 (both level-1 FP64).
// True when every case's load is rounding noise (e.g. the uniform solid):
// max_m ||f_m|| <= 1e-12 ||f_e||_F sqrt(n_e).
static bool zero_load(const Hier& h, const double* fnorm) {
  double fmax = 0;
  for (int c = 0; c < h.C; ++c) fmax = std::max(fmax, fnorm[c]);
  return fmax <= 1e-12 * h.fe_norm * std::sqrt((double)h.lv[0].n_e);
}

static void rel_residual64(Hier& h, const double* f, const double* u, double* r, double* rel,
                           double* fnorm_out, hipStream_t s, bool u_zero = false) {
  const int n = h.lv[0].n_n, C = h.C, D = h.D;
  if (u_zero)  // r = f - K 0
    launch_copy<double>(f, r, (size_t)n * h.Q, s);
  else
    apply<double>(h, 0, EPI_RESID, u, f, r, C, s);
  double* rr = h.red_out + 48;
  double* ff = h.red_out + 56;
  launch_dot<double>(r, r, n, C, D, h.red_partial, rr, s);
  launch_dot<double>(f, f, n, C, D, h.red_partial, ff, s);
  double rh[8], fh[8];
  host_dot(h, rr, C, rh, s);
  host_dot(h, ff, C, fh, s);
  double fmax = 0;
  for (int c = 0; c < C; ++c) fmax = std::max(fmax, std::sqrt(fh[c]));
  for (int c = 0; c < C; ++c) {
    double den = std::sqrt(fh[c]);
    if (den <= 1e-12 * fmax) den = fmax;
    rel[c] = den > 0 ? std::sqrt(rh[c]) / den : 0.0;
    if (fnorm_out) fnorm_out[c] = den;
  }
}

static double* scratch64(Hier& h, double** slot) {
  if (!*slot) *slot = h.alloc<double>((size_t)h.lv[0].n_n * h.Q);
  return *slot;
}

// ================================================================ build

static int ilog2_exact(int v) {
  int k = 0;
  while ((1 << k) < v) ++k;
  return (1 << k) == v ? k : -1;
}

// Phase timer for the build (GMT_TIMING=1 prints phase wall times to stderr).
struct PhaseTimer {
  bool on;
  hipStream_t s;
  std::chrono::steady_clock::time_point t0;
  explicit PhaseTimer(hipStream_t st) : on(std::getenv("GMT_TIMING") != nullptr), s(st), t0(std::chrono::steady_clock::now()) {}
  void mark(const char* what) {
    if (!on) return;
    (void)hipStreamSynchronize(s);
    auto t1 = std::chrono::steady_clock::now();
    fprintf(stderr, "[gmt build] %-12s %8.3f ms\n", what, std::chrono::duration<double, std::milli>(t1 - t0).count());
    t0 = t1;
  }
};

// rho (nullable): a density field (SIMP, App. F.3) on the N^3 voxels; its active
// set is rho > prune and `vox` is then that set (built by the caller)
static void build(Hier& h, const uint8_t* vox, hipStream_t s, const double* rho = nullptr) {
  PhaseTimer timer(s);
  const int N = h.N;
  const size_t n3 = (size_t)N * N * N;
  element_constants(h);
  h.density = rho != nullptr;
  const int D = h.D, M = 8 * D;
  h.Ke64 = h.alloc<double>(M * M);
  h.Ke32 = h.alloc<float>(M * M);
  h.fe64 = h.alloc<double>(M * h.C);
  GMT_HIP(hipMemcpyAsync(h.Ke64, h.Ke, M * M * sizeof(double), hipMemcpyHostToDevice, s));
  launch_convert<double, float>(h.Ke64, h.Ke32, M * M, s);
  GMT_HIP(hipMemcpyAsync(h.fe64, h.fe, M * h.C * sizeof(double), hipMemcpyHostToDevice, s));
  h.X064 = h.alloc<double>(M * h.C);
  GMT_HIP(hipMemcpyAsync(h.X064, h.X0, M * h.C * sizeof(double), hipMemcpyHostToDevice, s));
  double Ps[8][8][8];
  local_prolongation(Ps);
  h.Ps = h.alloc<double>(512);
  GMT_HIP(hipMemcpyAsync(h.Ps, Ps, 512 * sizeof(double), hipMemcpyHostToDevice, s));
  h.red_partial = h.alloc<double>((size_t)kRedBlocks * 64);
  h.red_out = h.alloc<double>(256);
  h.gauge_tmp64 = h.alloc<double>(32);
  h.gauge_tmp32 = h.alloc<float>(32);

  // temporary buffers (released with the hierarchy; small relative to the maps)
  int* flags = h.alloc<int>(n3);
  int* scr = h.alloc<int>(scan_scratch_ints(n3));
  int* d_total = h.alloc<int>(1);
  uint8_t* dmask = h.alloc<uint8_t>(n3 / 8 + 1);

  h.lv.resize(h.L);
  for (int l = 0; l < h.L; ++l) {
    LevelData& d = h.lv[l];
    d.N = N >> l;
    const size_t nl3 = (size_t)d.N * d.N * d.N;
    d.elem_map = h.alloc<int>(nl3);
    d.node_map = h.alloc<int>(nl3);
    if (l == 0) {
      launch_voxel_elem_flags(vox, n3, flags, s);
    } else {
      launch_coarsen_flags(h.lv[l - 1].elem_map, h.lv[l - 1].N, flags, dmask, s);
    }
    const int64_t ne = scan_compact(flags, nl3, nullptr, nullptr, scr, d_total, s);
    if (ne == 0) fail(GMT_E_INVAL, "empty active set");
    d.n_e = (int)ne;
    d.elem_lin = h.alloc<int>(ne);
    scan_compact(flags, nl3, d.elem_map, d.elem_lin, scr, d_total, s);
    if (l == 0) {
      // one rigid body: every solid voxel reachable through shared nodes (the
      // flags buffer holds the union-find parents of the n_e elements)
      const int ncomp = count_components(d.elem_lin, d.n_e, d.elem_map, d.N, flags, d_total, s);
      timer.mark("components");
      if (ncomp != 1)
        fail(GMT_E_INVAL,
             "the solid voxels form %d node-connected components; each could translate on its own and the "
             "solver pins one node: reduce the cell to one component",
             ncomp);
    }
    launch_node_flags(d.elem_map, d.N, flags, s);
    const int64_t nn = scan_compact(flags, nl3, nullptr, nullptr, scr, d_total, s);
    d.n_n = (int)nn;
    d.node_lin = h.alloc<int>(nn);
    scan_compact(flags, nl3, d.node_map, d.node_lin, scr, d_total, s);
    d.occ8 = h.alloc<uint8_t>(nn);
    launch_occ8(d.node_lin, d.n_n, d.elem_map, d.N, d.occ8, s);
    if (l >= 1) {
      d.cmask = h.alloc<uint8_t>(ne);
      launch_gather_cmask(d.elem_lin, d.n_e, dmask, d.cmask, s);
    }
    // a density hierarchy's level-2 matrices depend on the children's scales: per element
    d.kind = l == 0 ? KIND_SHARED : (l == 1 && !h.density ? KIND_TABLE : KIND_PERELEM);
  }
  if (h.density) {
    // per element rho and scale s = rho_min + rho^p, per node the octant scales
    LevelData& d = h.lv[0];
    d.erho = h.alloc<double>(d.n_e);
    d.escale = h.alloc<double>(d.n_e);
    launch_element_scale(d.elem_lin, d.n_e, rho, h.simp_p, h.simp_rho_min, d.erho, d.escale, s);
    d.oscale64 = h.alloc<double>((size_t)d.n_n * 8);
    d.oscale32 = h.alloc<float>((size_t)d.n_n * 8);
    launch_node_oscale(d.node_lin, d.n_n, d.elem_map, d.N, d.escale, d.oscale64, d.oscale32, s);
    double* ones = h.alloc<double>(d.n_e);
    launch_fill<double>(ones, d.n_e, 1.0, s);
    launch_dot<double>(d.escale, ones, d.n_e, 1, 1, h.red_partial, h.red_out, s);
    host_dot(h, h.red_out, 1, &h.scale_sum, s);
    h.release(ones);
  }

  // level 1: interior (occupancy 255) and boundary node lists; in a density
  // hierarchy every node goes through the scaled masked stencil (boundary list)
  {
    LevelData& d = h.lv[0];
    int* tmpmap = h.alloc<int>(d.n_n);
    if (h.density) {
      d.boundary = h.alloc<int>(d.n_n);
      d.n_bnd = d.n_n;
      launch_iota(d.boundary, d.n_n, s);
    }
    for (int full = 1; full >= 0 && !h.density; --full) {
      launch_occ_flags(d.occ8, d.n_n, full, flags, s);
      const int64_t cnt = scan_compact(flags, d.n_n, nullptr, nullptr, scr, d_total, s);
      int* list = cnt > 0 ? h.alloc<int>(cnt) : nullptr;
      if (cnt > 0) scan_compact(flags, d.n_n, tmpmap, list, scr, d_total, s);
      if (full) {
        d.interior = list;
        d.n_int = (int)cnt;
      } else {
        d.boundary = list;
        d.n_bnd = (int)cnt;
      }
    }
    // runs of consecutive interior nodes along x (chunks of at most kRun)
    if (d.n_int > 0) {
      launch_run_flags(d.interior, d.n_int, d.node_lin, d.N, flags, s);
      const int64_t nr = scan_compact(flags, d.n_int, nullptr, nullptr, scr, d_total, s);
      d.runs = h.alloc<int>(nr + 1);
      scan_compact(flags, d.n_int, tmpmap, d.runs, scr, d_total, s);
      const int sentinel = d.n_int;
      GMT_HIP(hipMemcpyAsync(d.runs + nr, &sentinel, sizeof(int), hipMemcpyHostToDevice, s));
      d.n_runs = (int)nr;
    }
    if (d.n_bnd > 0) {
      d.bnd_nbrs = h.alloc<int>((size_t)d.n_bnd * kBndStride);
      if (reinterpret_cast<uintptr_t>(d.bnd_nbrs) % 16 != 0)  // the sweeps read its rows as int4
        fail(GMT_E_STATE, "boundary neighbour table is not 16-byte aligned");
      launch_boundary_nbrs(d.boundary, d.n_bnd, d.node_lin, d.node_map, d.N, d.bnd_nbrs, s);
    }
    // tables of the staged interior sweep: distinct neighbour ids per group of
    // nb interior nodes (counted first; written for the groups within the FP32
    // cap); per precision, the groups within its cap are staged, the others'
    // nodes listed for the plain kernel
    if (d.n_int > 0) {
      // GMT_STAGE_NODES=256|512 pins the group size (tests of both on small cells)
      const char* env_nb = std::getenv("GMT_STAGE_NODES");
      const int nb = env_nb && *env_nb ? (std::atoi(env_nb) == 512 ? 512 : 256) : (d.n_int >= kStageBigFrom ? 512 : 256);
      int cap32 = nb * stage_k(nb, false), cap64 = nb * stage_k(nb, true);
      // GMT_STAGE_CAP=<k> lowers both caps (tests of the unstaged remainder)
      if (const char* ec = std::getenv("GMT_STAGE_CAP"))
        if (*ec && std::atoi(ec) > 0) cap32 = std::min(cap32, std::atoi(ec)), cap64 = std::min(cap64, std::atoi(ec));
      d.st_nodes = nb;
      const int nblk = (d.n_int + nb - 1) / nb;
      int* cnt = h.alloc<int>(nblk);
      launch_stage_tables(d.interior, d.n_int, d.node_lin, d.node_map, d.N, nb, 0, nullptr, 0, cnt, nullptr, nullptr,
                          nullptr, s);
      std::vector<int> hc(nblk);
      GMT_HIP(hipMemcpyAsync(hc.data(), cnt, nblk * sizeof(int), hipMemcpyDeviceToHost, s));
      GMT_HIP(hipStreamSynchronize(s));
      auto nodes_of = [&](int b) { return std::min(nb, d.n_int - nb * b); };
      std::vector<long long> ho(nblk + 1, 0);
      std::vector<int> good[2], rest[2];
      for (int b = 0; b < nblk; ++b) {
        ho[b + 1] = ho[b] + (hc[b] <= cap32 ? hc[b] : 0);
        (hc[b] <= cap32 ? good[0] : rest[0]).push_back(b);
        (hc[b] <= cap64 ? good[1] : rest[1]).push_back(b);
      }
      if (!good[0].empty()) {
        int* g32 = h.alloc<int>(good[0].size());
        d.st_off = h.alloc<long long>(ho.size());
        d.st_ids = h.alloc<int>((size_t)std::max(ho.back(), 1LL));
        d.st_slot = h.alloc<uint16_t>((size_t)d.n_int * kSlotStride);
        GMT_HIP(hipMemcpyAsync(g32, good[0].data(), good[0].size() * sizeof(int), hipMemcpyHostToDevice, s));
        GMT_HIP(hipMemcpyAsync(d.st_off, ho.data(), ho.size() * sizeof(long long), hipMemcpyHostToDevice, s));
        launch_stage_tables(d.interior, d.n_int, d.node_lin, d.node_map, d.N, nb, 1, g32, (int)good[0].size(), cnt,
                            d.st_off, d.st_ids, d.st_slot, s);
        d.st_blk32 = g32;
        d.n_st_blk32 = (int)good[0].size();
        if (!good[1].empty()) {
          d.st_blk64 = h.alloc<int>(good[1].size());
          GMT_HIP(hipMemcpyAsync(d.st_blk64, good[1].data(), good[1].size() * sizeof(int), hipMemcpyHostToDevice, s));
          d.n_st_blk64 = (int)good[1].size();
        }
      }
      for (int p = 0; p < 2; ++p) {
        if (rest[p].empty()) continue;
        long long nr = 0;
        for (int b : rest[p]) nr += nodes_of(b);
        int* rb = h.alloc<int>(rest[p].size());
        GMT_HIP(hipMemcpyAsync(rb, rest[p].data(), rest[p].size() * sizeof(int), hipMemcpyHostToDevice, s));
        int* list = h.alloc<int>((size_t)rest[p].size() * nb);
        launch_gather_blocks(d.interior, d.n_int, nb, rb, (int)rest[p].size(), list, s);
        GMT_HIP(hipStreamSynchronize(s));
        h.release(rb);
        (p == 0 ? d.st_rest32 : d.st_rest64) = list;
        (p == 0 ? d.n_st_rest32 : d.n_st_rest64) = (int)nr;
      }
      GMT_HIP(hipStreamSynchronize(s));
      h.release(cnt);
    }
    GMT_HIP(hipStreamSynchronize(s));
    h.release(tmpmap);
  }
  // assembled interior stencil of the shared K_e: S[j][d][d2] over the 27 offsets
  {
    std::vector<double> S((size_t)27 * D * D, 0.0);
    for (int k = 0; k < 8; ++k) {
      const int a = 7 - k;
      for (int m = 0; m < 8; ++m) {
        const int j = ((k & 1) + (m & 1)) + 3 * (((k >> 1) & 1) + ((m >> 1) & 1)) +
                      9 * (((k >> 2) & 1) + ((m >> 2) & 1));
        for (int d = 0; d < D; ++d)
          for (int d2 = 0; d2 < D; ++d2) S[(j * D + d) * D + d2] += h.Ke[(a * D + d) * M + m * D + d2];
      }
    }
    double smax = 0;
    for (double v : S) smax = std::max(smax, std::fabs(v));
    for (int j = 0; j < 27; ++j) {
      const int o[3] = {j % 3 - 1, (j / 3) % 3 - 1, j / 9 - 1};
      for (int d = 0; d < D; ++d)
        for (int d2 = 0; d2 < D; ++d2) {
          const bool nz = D == 1 ? ((o[0] != 0) + (o[1] != 0) + (o[2] != 0)) != 1
                                 : (d == d2 || (o[d] != 0 && o[d2] != 0));
          if (!nz && std::fabs(S[(j * D + d) * D + d2]) > 1e-12 * smax)
            fail(GMT_E_STATE, "interior stencil entry (%d,%d,%d) expected zero", j, d, d2);
        }
    }
    // symmetry-class values of K_e (taken from block row 0, where the sign is
    // +1), then every entry of K_e checked against its class value
    const int NK = D == 1 ? 4 : 14;
    std::vector<double> kc(NK, 0.0);
    std::vector<char> have(NK, 0);
    double kmax = 0;
    for (int r = 0; r < M * M; ++r) kmax = std::max(kmax, std::fabs(h.Ke[r]));
    auto cls = [&](int delta, int d, int d2) {
      return D == 1 ? kcls_index<1>(delta, d, d2) : kcls_index<3>(delta, d, d2);
    };
    for (int m = 0; m < 8; ++m)
      for (int d = 0; d < D; ++d)
        for (int d2 = 0; d2 < D; ++d2) {
          const int c = cls(m, d, d2);
          if (!have[c]) kc[c] = h.Ke[d * M + m * D + d2], have[c] = 1;
        }
    for (int a = 0; a < 8; ++a)
      for (int m = 0; m < 8; ++m)
        for (int d = 0; d < D; ++d)
          for (int d2 = 0; d2 < D; ++d2) {
            const bool neg = D == 1 ? kcls_negative<1>(a, d, d2) : kcls_negative<3>(a, d, d2);
            const double v = (neg ? -1.0 : 1.0) * h.Ke[(a * D + d) * M + m * D + d2];
            if (std::fabs(v - kc[cls(a ^ m, d, d2)]) > 1e-12 * kmax)
              fail(GMT_E_STATE, "K_e entry (%d,%d,%d,%d) is not its symmetry-class value", a, m, d, d2);
          }
    // symmetry-class values of S, and every stencil entry checked against them
    const int NS = D == 1 ? 4 : 8;
    std::vector<double> sc(NS, 0.0);
    std::vector<char> shave(NS, 0);
    auto scl = [&](int j, int d, int d2) {
      return D == 1 ? scls_index<1>(j, d, d2) : scls_index<3>(j, d, d2);
    };
    auto sneg = [&](int j, int d, int d2) {
      return D == 1 ? scls_negative<1>(j, d, d2) : scls_negative<3>(j, d, d2);
    };
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < 27; ++j)
        for (int d = 0; d < D; ++d)
          for (int d2 = 0; d2 < D; ++d2) {
            const int o[3] = {j % 3 - 1, (j / 3) % 3 - 1, j / 9 - 1};
            const double v = S[(j * D + d) * D + d2];
            const bool zero = D == 3 && d != d2 && o[d] * o[d2] == 0;
            if (zero) continue;  // a structural zero (checked above)
            const double w = (sneg(j, d, d2) ? -1.0 : 1.0) * v;
            const int c = scl(j, d, d2);
            if (pass == 0) {
              if (!shave[c]) sc[c] = w, shave[c] = 1;
            } else if (std::fabs(w - sc[c]) > 1e-12 * smax) {
              fail(GMT_E_STATE, "stencil entry (%d,%d,%d) is not its symmetry-class value", j, d, d2);
            }
          }
    h.scls64 = h.alloc<double>(NS);
    h.scls32 = h.alloc<float>(NS);
    GMT_HIP(hipMemcpyAsync(h.scls64, sc.data(), NS * sizeof(double), hipMemcpyHostToDevice, s));
    launch_convert<double, float>(h.scls64, h.scls32, NS, s);
    h.kcls64 = h.alloc<double>(NK);
    h.kcls32 = h.alloc<float>(NK);
    GMT_HIP(hipMemcpyAsync(h.kcls64, kc.data(), NK * sizeof(double), hipMemcpyHostToDevice, s));
    launch_convert<double, float>(h.kcls64, h.kcls32, NK, s);
    h.S64 = h.alloc<double>(S.size());
    h.S32 = h.alloc<float>(S.size());
    GMT_HIP(hipMemcpyAsync(h.S64, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice, s));
    launch_convert<double, float>(h.S64, h.S32, S.size(), s);
    GMT_HIP(hipStreamSynchronize(s));
  }
  timer.mark("maps");
  // Galerkin operators
  if (h.L >= 2) {
    std::vector<double> tab;
    mask_table(h, Ps, tab);
    h.table64 = h.alloc<double>(tab.size());
    h.table32 = h.alloc<float>(tab.size());
    GMT_HIP(hipMemcpyAsync(h.table64, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, s));
    launch_convert<double, float>(h.table64, h.table32, tab.size(), s);
    GMT_HIP(hipStreamSynchronize(s));
  }
  for (int l = h.density ? 1 : 2; l < h.L; ++l) {
    LevelData& d = h.lv[l];
    const LevelData& f = h.lv[l - 1];
    d.Kel64 = h.alloc<double>((size_t)d.n_e * M * M);
    d.Kel32 = h.alloc<float>((size_t)d.n_e * M * M);
    const double* src = f.kind == KIND_SHARED ? h.Ke64 : (f.kind == KIND_TABLE ? h.table64 : f.Kel64);
    launch_galerkin(d.elem_lin, d.n_e, d.N, f.elem_map, f.cmask, src, f.kind, D, h.Ps,
                    l == 1 ? h.lv[0].escale : nullptr, d.Kel64, d.Kel32, s);
  }
  timer.mark("galerkin");
  // Jacobi diagonals
  for (int l = 0; l < h.L; ++l) {
    LevelData& d = h.lv[l];
    const size_t nd = (size_t)d.n_n * D;
    d.diag64 = h.alloc<double>(nd);
    d.dinv64 = h.alloc<double>(nd);
    d.dinv32 = h.alloc<float>(nd);
    launch_diagonal<double>(h.view<double>(l), d.kind, D, d.diag64, s);
    launch_inv<double>(d.diag64, d.dinv64, nd, s);
    launch_convert<double, float>(d.dinv64, d.dinv32, nd, s);
  }
  // load vector
  h.f64 = h.alloc<double>((size_t)h.lv[0].n_n * h.Q);
  launch_load_vector(h.lv[0].node_lin, h.lv[0].occ8, h.lv[0].oscale64, h.lv[0].n_n, D, h.C, h.fe64, h.f64, s);

  timer.mark("diag+load");
  EventSet evs;
  CoarseHost ch;
  coarse_fetch(h, s, ch, evs);
  void* pw[7] = {};
  // lambda_max(D^-1 K) per level by power iteration. The iterate only has to
  // point at the top of the spectrum, so the iterations run in FP32 (half the
  // operator bytes); the Rayleigh quotient that becomes the estimate is taken in
  // FP64, so the estimate stays below lambda_max up to FP64 rounding.  The
  // levels are independent and their sweeps short (one vector, latency-bound
  // on the coarse levels): level 1 runs on s, the others on auxiliary streams
  // forked from s by an event and joined back before the host reads the
  // quotients.  Each level has buffers and reduction slots of its own.
  {
    const int iters = h.p.power_iters > 0 ? h.p.power_iters : 20;
    std::vector<size_t> off(h.L + 1, 0);
    for (int l = 0; l < h.L; ++l) off[l + 1] = off[l] + ((size_t)h.lv[l].n_n * D + 63) / 64 * 64;
    float* X32 = h.alloc<float>(off[h.L]);  // released after the stream sync below
    float* Y32 = h.alloc<float>(off[h.L]);
    float* T32 = h.alloc<float>(off[h.L]);
    double* X64 = h.alloc<double>(off[h.L]);
    double* Y64 = h.alloc<double>(off[h.L]);
    double* T64 = h.alloc<double>(off[h.L]);
    double* part = h.alloc<double>((size_t)h.L * kRedBlocks);
    pw[0] = X32, pw[1] = Y32, pw[2] = T32, pw[3] = X64, pw[4] = Y64, pw[5] = T64, pw[6] = part;
    double* o = h.red_out + 64;  // [4 + 2l, 5 + 2l]: quotient of level l; [40 + l]: its norm
    // One vector: on level 1 the class-assembled boundary sweep (cb 7, or 9
    // with the staged interior) costs in proportion to the number of cases,
    // the masked-stencil one (cb 0, the default before the autotuner runs)
    // does not.
    const int cb_keep = h.lv[0].cb32, cb_keep64 = h.lv[0].cb64;
    if (h.lv[0].kind == KIND_SHARED) h.lv[0].cb32 = h.lv[0].cb64 = h.lv[0].n_st_blk32 > 0 ? 9 : 7;
    hipEvent_t fork = evs.make();
    GMT_HIP(hipEventRecord(fork, s));
    for (int l = 0; l < h.L; ++l) {
      LevelData& d = h.lv[l];
      const int n = d.n_n;
      const size_t nd = (size_t)n * D;
      hipStream_t sl = s;
      if (l > 0) {
        sl = aux_stream(l - 1);
        GMT_HIP(hipStreamWaitEvent(sl, fork, 0));
      }
      float* x32 = X32 + off[l];
      float* y32 = Y32 + off[l];
      float* t32 = T32 + off[l];
      double* x = X64 + off[l];
      double* y = Y64 + off[l];
      double* t = T64 + off[l];
      double* pl = part + (size_t)l * kRedBlocks;
      double* nrm = o + 40 + l;
      launch_random(x, nd, h.p.seed + 0x1000193ull * (l + 1), sl);
      launch_convert<double, float>(x, x32, nd, sl);
      // x <- D^-1 K x, normalised on the device (no host round trip) every
      // fourth step and after the last; D^-1 K has eigenvalues of order one, so
      // four unnormalised steps stay far inside the FP32 range.
      for (int it = 0; it < iters; ++it) {
        apply<float>(h, l, EPI_KU, x32, nullptr, y32, 1, sl);
        launch_smooth_zero<float>(n, D, 1, y32, d.dinv32, 1.0f, t32, nullptr, sl);  // t = D^-1 K x
        if ((it + 1) % 4 == 0 || it + 1 == iters) {
          launch_dot<float>(t32, t32, n, 1, D, pl, nrm, sl);
          launch_normalize<float>(t32, nd, nrm, x32, sl);
        } else {
          std::swap(x32, t32);
        }
      }
      launch_convert<float, double>(x32, x, nd, sl);
      // Rayleigh quotient x.Kx / x.Dx (a lower bound of lambda_max)
      apply<double>(h, l, EPI_KU, x, nullptr, y, 1, sl);
      launch_smooth_zero<double>(n, D, 1, x, d.diag64, 1.0, t, nullptr, sl);  // t = D x
      launch_dot<double>(x, y, n, 1, D, pl, o + 4 + 2 * l, sl);
      launch_dot<double>(x, t, n, 1, D, pl, o + 5 + 2 * l, sl);
      if (l > 0) {
        hipEvent_t done = evs.make();
        GMT_HIP(hipEventRecord(done, sl));
        GMT_HIP(hipStreamWaitEvent(s, done, 0));
      }
    }
    h.lv[0].cb32 = cb_keep;
    h.lv[0].cb64 = cb_keep64;
    // the host factors the coarsest operator while the iterations run
    coarse_factor(h, s, ch);
    // one host round trip for the quotients of all levels
    double hv[2 * 12];
    host_dot(h, o + 4, 2 * h.L, hv, s);
    for (int l = 0; l < h.L; ++l) {
      const double lam = hv[2 * l + 1] > 0 ? hv[2 * l] / hv[2 * l + 1] : 0.0;
      if (!(lam > 0) || !std::isfinite(lam)) fail(GMT_E_SINGULAR, "lambda_max estimate failed on level %d", l + 1);
      h.lv[l].lam = lam;
    }
  }
  timer.mark("lambda+coarse");
  GMT_HIP(hipStreamSynchronize(s));
  for (void* b : pw) h.release(b);
  h.release(flags);
  h.release(scr);
  h.release(d_total);
  h.release(dmask);
}

// ================================================================ solve

// An FP32 inner solve that needs more than this many iterations marks an
// ill-conditioned cell (thin, nearly mechanism-like members), where the FP32
// recurrence drifts from the true residual and each refinement step gains
// little: such a cell needs about three times as many FP32 iterations as FP64
// ones in total, so it continues with the FP64 recurrence.
constexpr int kMaxInner32 = 120;
// inner-solve mode after such a switch: FP64 Krylov recurrence and K.p, FP32
// V-cycle (pcg<double, true>)
constexpr int kInnerMixed = 100;

// Mixed precision runs only a few level-1 FP64 residual sweeps: rather than
// timing the FP64 candidates for them, they borrow the launch shape the FP32
// autotuner chose for level 1 (every variant exists in both precisions).  A
// later FP64 autotune (FP64 inner solves) still times its own.
static void borrow_f32_shape(Hier& h) {
  LevelData& d = h.lv[0];
  if (d.tuned64 || !d.tuned32) return;
  d.bs64 = d.bs32;
  d.cb64 = d.cb32;
  d.xcd64 = d.xcd32;
}

static void solve(Hier& h, const double* f, double* u, const gmt_solve_opts* o, gmt_solve_report* rep,
                  hipStream_t s, gmt_status* st, bool u_zero = false) {
  const double tol = o && o->tol > 0 ? o->tol : 1e-5;
  const int max_iter = o && o->max_iter > 0 ? o->max_iter : 500;
  const int max_outer = o && o->max_outer > 0 ? o->max_outer : 8;  // (+ one FP64 fallback switch)
  const int prec = o ? o->precision : GMT_F64;
  const int check = o && o->check_every > 0 ? o->check_every : 1;
  const bool graph = o && o->graph;
  if (prec != GMT_F64 && prec != GMT_F32) fail(GMT_E_INVAL, "bad precision");
  // GMT_MAX_INNER32=<k> lowers the FP32 inner-iteration cap (tests use it to
  // reach the FP64-recurrence path on small cells)
  int max_inner32 = kMaxInner32;
  if (const char* e = std::getenv("GMT_MAX_INNER32"))
    if (*e && std::atoi(e) > 0) max_inner32 = std::min(kMaxInner32, std::atoi(e));
  const CycleCfg cfg = make_cycle(h, o ? &o->cycle : nullptr);
  if (cfg.schedule == GMT_CYCLE_F)
    fail(GMT_E_INVAL, "the F-cycle is not symmetric: it cannot precondition conjugate gradients");
  double* r64 = scratch64(h, &h.s_r64);
  if (prec == GMT_F32) {
    autotune<float>(h, s);
    borrow_f32_shape(h);
  } else {
    autotune<double>(h, s);
  }
  const int C = h.C;
  const size_t tot = (size_t)h.lv[0].n_n * h.Q;
  gmt_solve_report R{};
  R.c = C;
  double rel[8], den[8];
  int its = 0;
  int inner_prec = prec;          // precision of the next inner solve
  bool last_f32 = false;          // the last accepted update came from an FP32 inner solve
  bool stalled32 = false;         // an FP32 inner solve stopped on stagnation
  double prev_worst = INFINITY;
  for (int outer = 0;; ++outer) {
    rel_residual64(h, f, u, r64, rel, den, s, outer == 0 && u_zero);
    if (outer == 0 && zero_load(h, den)) {
      // zero load: the solution in the pinned gauge is u = 0
      launch_fill<double>(u, tot, 0.0, s);
      for (int c = 0; c < C; ++c) rel[c] = 0.0;
    }
    double worst = 0;
    for (int c = 0; c < C; ++c) {
      if (!std::isfinite(rel[c])) worst = INFINITY;
      else worst = std::max(worst, rel[c]);
      R.rel_res[c] = rel[c];
      if (outer == 0) R.rel_res_init[c] = rel[c];
    }
    if (outer == 0 && !(worst <= 1.0)) {
      // the initial guess is not finite or is farther from the solution than
      // zero (the zero guess has residual ||f||): start from zero instead
      launch_fill<double>(u, tot, 0.0, s);
      rel_residual64(h, f, u, r64, rel, den, s);
      worst = 0;
      for (int c = 0; c < C; ++c) {
        worst = std::isfinite(rel[c]) ? std::max(worst, rel[c]) : INFINITY;
        R.rel_res[c] = rel[c];
      }
    }
    R.outer = outer + 1;
    if (worst <= tol) {
      R.converged = 1;
      break;
    }
    if (stalled32 && inner_prec == GMT_F32 && worst < 0.5 * prev_worst) {
      inner_prec = kInnerMixed;  // FP64 Krylov, FP32 V-cycle
      last_f32 = false;
    }
    if (last_f32 && !(worst < 0.5 * prev_worst)) {
      // the FP32 inner solve did not halve the FP64 residual (an ill-conditioned
      // cell where the FP32 recurrence stalls or diverges): undo that update and
      // finish with the FP64 recurrence (FP32 V-cycle); the iterate before the
      // step was kept, so the undo is exact
      launch_copy<double>(h.s_usave, u, tot, s);
      inner_prec = kInnerMixed;
      last_f32 = false;
      rel_residual64(h, f, u, r64, rel, den, s);
      worst = 0;
      for (int c = 0; c < C; ++c) {
        worst = std::isfinite(rel[c]) ? std::max(worst, rel[c]) : INFINITY;
        R.rel_res[c] = rel[c];
      }
    }
    if (!std::isfinite(worst) || outer >= max_outer || its >= max_iter) break;
    prev_worst = worst;
    double itol[8];
    // an FP32 inner solve is asked for at most four orders of reduction; the
    // FP64 refinement step recovers the rest
    const double floor = inner_prec == GMT_F32 ? 1e-4 : 1e-14;
    for (int c = 0; c < C; ++c) {
      // target ||r_m|| <= tol/2 * den_m after this step; relative to the current ||r_m||
      const double rn = rel[c] * den[c];
      double t = rn > 0 ? 0.5 * tol * den[c] / rn : 1.0;
      itol[c] = std::min(0.9, std::max(floor, t));
    }
    if (inner_prec == GMT_F32) {
      if (!h.s_b32) h.s_b32 = h.alloc<float>(tot);
      if (!h.s_x32) h.s_x32 = h.alloc<float>(tot);
      launch_convert<double, float>(r64, h.s_b32, tot, s);
      bool reached = false;
      its += pcg<float>(h, h.s_b32, h.s_x32, itol, std::min(max_iter - its, max_inner32), check, graph, cfg, s,
                        &reached);
      launch_copy<double>(u, scratch64(h, &h.s_usave), tot, s);
      launch_accumulate<float>(u, h.s_x32, tot, s, 1.0);
      last_f32 = true;
      // an FP32 inner solve that stalled, or ran into kMaxInner32, short of its
      // target: keep its update (checked above on the next pass) and take FP64
      // inner solves from here
      if (!reached && its < max_iter) stalled32 = true;
    } else if (inner_prec == kInnerMixed) {
      autotune<double>(h, s);
      double* x64 = scratch64(h, &h.s_x64);
      its += pcg<double, true>(h, r64, x64, itol, max_iter - its, check, graph, cfg, s);
      launch_accumulate<double>(u, x64, tot, s, 1.0);
      last_f32 = false;
    } else {
      if (prec == GMT_F32) autotune<double>(h, s);
      double* x64 = scratch64(h, &h.s_x64);
      its += pcg<double>(h, r64, x64, itol, max_iter - its, check, graph, cfg, s);
      launch_accumulate<double>(u, x64, tot, s, 1.0);
      last_f32 = false;
    }
  }
  if (h.p.gauge == 1)
    launch_project<double>(u, h.lv[0].n_n, h.Q, h.D, h.red_partial, h.red_out + 200, s);
  else
    launch_gauge_shift<double>(u, h.lv[0].n_n, h.Q, h.D, h.gauge_tmp64, s);
  GMT_HIP(hipStreamSynchronize(s));
  R.iterations = its;
  if (rep) *rep = R;
  *st = R.converged ? GMT_OK : GMT_E_NOCONV;
  if (!R.converged) {
    double worst = 0;
    for (int c = 0; c < C; ++c) worst = std::max(worst, R.rel_res[c]);
    g_last_error = "gmt_solve: tolerance not reached (residual " + std::to_string(worst) + " after " +
                   std::to_string(its) + " iterations)";
  }
}

}  // namespace gmt

// ================================================================ C ABI

using namespace gmt;

struct gmt_hier {
  Hier h;
};

static hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

static void check_level(const gmt_hier* H, int level) {
  if (!H) fail(GMT_E_INVAL, "null hierarchy");
  if (level < 1 || level > H->h.L) fail(GMT_E_INVAL, "level %d outside 1..%d", level, H->h.L);
}

static void check_dtype(int dtype) {
  if (dtype != GMT_F64 && dtype != GMT_F32) fail(GMT_E_INVAL, "dtype must be GMT_F64 or GMT_F32");
}

// Every gmt_* definition below has C linkage through its declaration in gmt.h.

const char* gmt_last_error(void) { return g_last_error.c_str(); }

template <typename T>
static double time_sweep(Hier& h, int l, int reps, hipStream_t s) {
  autotune<T>(h, s);  // time the launch shape the solver uses
  h.ensure_io<T>(l);
  Work<T>& W = h.work<T>();
  const size_t n = (size_t)h.lv[l].n_n * h.Q;
  T* f = W.io1[l];
  T* u = W.io2[l];
  T* alt = W.io3[l];
  launch_fill<T>(f, n, T(1), s);
  launch_fill<T>(u, n, T(0), s);
  launch_fill<T>(W.dvec[l], n, T(0), s);
  const double lam = h.lv[l].lam;
  const double lo = lam / 30.0, hi = 1.1 * lam;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  const double rn = 1.0 / (2.0 * sigma - 1.0 / sigma);
  auto sweep = [&]() {
    apply<T>(h, l, EPI_CHEB, u, f, alt, h.C, s, T(0), (T)(rn / sigma), (T)(2.0 * rn / delta), W.dvec[l]);
    std::swap(u, alt);
  };
  for (int k = 0; k < 2; ++k) sweep();
  hipEvent_t e0, e1;
  GMT_HIP(hipEventCreate(&e0));
  GMT_HIP(hipEventCreate(&e1));
  GMT_HIP(hipEventRecord(e0, s));
  for (int k = 0; k < reps; ++k) sweep();
  GMT_HIP(hipEventRecord(e1, s));
  GMT_HIP(hipEventSynchronize(e1));
  float ms = 0;
  GMT_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

gmt_status gmt_time_sweep(gmt_hier_t H, int32_t level, int32_t reps, int32_t dtype, double* h_ms, void* stream) {
  return guarded([&] {
    check_level(H, level);
    check_dtype(dtype);
    if (!h_ms) fail(GMT_E_INVAL, "h_ms is NULL");
    if (reps < 1 || reps > 100000) fail(GMT_E_INVAL, "reps out of range");
    *h_ms = dtype == GMT_F64 ? time_sweep<double>(H->h, level - 1, reps, S(stream))
                             : time_sweep<float>(H->h, level - 1, reps, S(stream));
  });
}

// Validates the parameters and sets up the hierarchy object (no device work).
static gmt_hier* new_hierarchy(int32_t N, const gmt_params* params) {
  if (!params) fail(GMT_E_INVAL, "params is NULL");
  if (N < 2 || N > 1024) fail(GMT_E_INVAL, "N = %d outside 2..1024", N);
  const int L = params->levels;
  if (L < 1 || L > 12) fail(GMT_E_INVAL, "levels = %d outside 1..12", L);
  if (N % (1 << (L - 1)) != 0 || (N >> (L - 1)) < 2)
    fail(GMT_E_INVAL, "N = %d must be divisible by 2^(L-1) = %d with N_L >= 2", N, 1 << (L - 1));
  if (params->physics != GMT_ELASTIC && params->physics != GMT_THERMAL) fail(GMT_E_INVAL, "bad physics");
  if ((params->alloc == nullptr) != (params->release == nullptr))
    fail(GMT_E_INVAL, "alloc and release must be given together");
  if (params->gauge != 0 && params->gauge != 1) fail(GMT_E_INVAL, "gauge must be 0 (node 0 pinned) or 1 (zero mean)");
  gmt_hier* H = new gmt_hier();
  Hier& h = H->h;
  h.p = *params;
  if (h.p.E == 0) h.p.E = 1.0;
  if (h.p.nu == 0 && params->physics == GMT_ELASTIC) h.p.nu = 0.3;
  if (h.p.kappa == 0) h.p.kappa = 1.0;
  if (h.p.physics == GMT_ELASTIC && !(h.p.E > 0 && h.p.nu > -1.0 && h.p.nu < 0.5)) {
    delete H;
    fail(GMT_E_INVAL, "need E > 0 and -1 < nu < 0.5");
  }
  if (h.p.physics == GMT_THERMAL && !(h.p.kappa > 0)) {
    delete H;
    fail(GMT_E_INVAL, "need kappa > 0");
  }
  h.N = N;
  h.L = L;
  h.D = params->physics == GMT_ELASTIC ? 3 : 1;
  h.C = params->physics == GMT_ELASTIC ? 6 : 3;
  h.Q = h.C * h.D;
  return H;
}

gmt_status gmt_build_hierarchy(const uint8_t* d_voxels, int32_t N, const gmt_params* params, void* stream,
                               gmt_hier_t* out) {
  gmt_hier* H = nullptr;
  gmt_status st = guarded([&] {
    if (!out) fail(GMT_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!d_voxels) fail(GMT_E_INVAL, "voxels is NULL");
    H = new_hierarchy(N, params);
    (void)ilog2_exact;
    build(H->h, d_voxels, S(stream));
    GMT_HIP(hipStreamSynchronize(S(stream)));
    *out = H;
  });
  if (st != GMT_OK && H) {
    (void)hipDeviceSynchronize();
    H->h.release_all();
    delete H;
  }
  return st;
}

gmt_status gmt_build_density_hierarchy(const double* d_rho, int32_t N, const gmt_simp_params* sp,
                                       const gmt_params* params, void* stream, gmt_hier_t* out) {
  gmt_hier* H = nullptr;
  gmt_status st = guarded([&] {
    if (!out) fail(GMT_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!d_rho || !sp) fail(GMT_E_INVAL, "null pointer");
    if (!(sp->p >= 1.0) || !(sp->rho_min > 0.0) || !(sp->prune >= 0.0) || !(sp->prune < 1.0))
      fail(GMT_E_INVAL, "need p >= 1, rho_min > 0 and 0 <= prune < 1");
    if (params && params->levels < 2) fail(GMT_E_INVAL, "a density hierarchy needs at least 2 levels");
    H = new_hierarchy(N, params);
    Hier& h = H->h;
    h.simp_p = sp->p;
    h.simp_rho_min = sp->rho_min;
    h.simp_prune = sp->prune;
    hipStream_t s = S(stream);
    const size_t n3 = (size_t)N * N * N;
    uint8_t* vox = h.alloc<uint8_t>(n3);
    launch_density_flags(d_rho, n3, sp->prune, vox, s);
    build(h, vox, s, d_rho);
    GMT_HIP(hipStreamSynchronize(s));
    h.release(vox);
    *out = H;
  });
  if (st != GMT_OK && H) {
    (void)hipDeviceSynchronize();
    H->h.release_all();
    delete H;
  }
  return st;
}

void gmt_destroy(gmt_hier_t H) {
  if (!H) return;
  (void)hipDeviceSynchronize();
  nn_release(H->h);
  H->h.release_graphs();
  H->h.release_all();
  delete H;
}

gmt_status gmt_level_info(gmt_hier_t H, int32_t level, gmt_level_desc* out) {
  return guarded([&] {
    check_level(H, level);
    if (!out) fail(GMT_E_INVAL, "out is NULL");
    const LevelData& d = H->h.lv[level - 1];
    out->N = d.N;
    out->n_e = d.n_e;
    out->n_n = d.n_n;
    out->c = H->h.C;
    out->d = H->h.D;
    out->lambda_max = d.lam;
    out->sweep_variant[0] = d.cb32;
    out->sweep_variant[1] = d.cb64;
    out->sweep_block[0] = d.bs32;
    out->sweep_block[1] = d.bs64;
    out->sweep_xcd[0] = d.xcd32;
    out->sweep_xcd[1] = d.xcd64;
  });
}

gmt_status gmt_export_maps(gmt_hier_t H, int32_t level, int32_t* d_elem_lin, int32_t* d_node_lin, uint8_t* d_occ8,
                           int32_t* d_elem_nodes, int32_t* d_prol_idx, double* d_prol_w, void* stream) {
  return guarded([&] {
    check_level(H, level);
    Hier& h = H->h;
    const LevelData& d = h.lv[level - 1];
    hipStream_t s = S(stream);
    if (d_elem_lin) GMT_HIP(hipMemcpyAsync(d_elem_lin, d.elem_lin, d.n_e * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (d_node_lin) GMT_HIP(hipMemcpyAsync(d_node_lin, d.node_lin, d.n_n * sizeof(int), hipMemcpyDeviceToDevice, s));
    if (d_occ8) GMT_HIP(hipMemcpyAsync(d_occ8, d.occ8, d.n_n, hipMemcpyDeviceToDevice, s));
    if (d_elem_nodes) launch_elem_nodes(d.elem_lin, d.n_e, d.node_map, d.N, d_elem_nodes, s);
    if (d_prol_idx || d_prol_w) {
      if (level == h.L) fail(GMT_E_INVAL, "no transfer stencil below the coarsest level");
      const LevelData& c = h.lv[level];
      launch_prol_maps(d.node_lin, d.n_n, d.N, c.node_map, c.N, d_prol_idx, d_prol_w, s);
    }
  });
}

gmt_status gmt_export_element_matrices(gmt_hier_t H, int32_t level, double* d_K, void* stream) {
  return guarded([&] {
    check_level(H, level);
    if (!d_K) fail(GMT_E_INVAL, "d_K is NULL");
    Hier& h = H->h;
    const LevelData& d = h.lv[level - 1];
    if (h.density && level == 1)
      fail(GMT_E_INVAL, "level-1 matrices of a density hierarchy are s_e K0: export levels >= 2");
    launch_expand_elem_matrices(h.view<double>(level - 1), d.kind, d.n_e, h.D, d.elem_lin, d_K, S(stream));
  });
}

gmt_status gmt_export_diagonal(gmt_hier_t H, int32_t level, double* d_D, void* stream) {
  return guarded([&] {
    check_level(H, level);
    if (!d_D) fail(GMT_E_INVAL, "d_D is NULL");
    const LevelData& d = H->h.lv[level - 1];
    GMT_HIP(hipMemcpyAsync(d_D, d.diag64, (size_t)d.n_n * H->h.D * sizeof(double), hipMemcpyDeviceToDevice,
                           S(stream)));
  });
}

gmt_status gmt_load_vector(gmt_hier_t H, void* d_f, int32_t dtype, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    check_dtype(dtype);
    if (!d_f) fail(GMT_E_INVAL, "d_f is NULL");
    Hier& h = H->h;
    const int n = h.lv[0].n_n;
    if (dtype == GMT_F64)
      launch_soa_to_aos<double, double>(h.f64, (double*)d_f, n, h.C, h.D, S(stream));
    else
      launch_soa_to_aos<double, float>(h.f64, (float*)d_f, n, h.C, h.D, S(stream));
  });
}

// ABI vectors are [n][c][d]; the solver's are [c*d + d][n].  The staging helpers
// below move one caller vector of level l into / out of a level-l work buffer.
template <typename T>
static T* stage_in(Hier& h, int l, const void* src, T* dst, hipStream_t s) {
  launch_aos_to_soa<T, T>((const T*)src, dst, h.lv[l].n_n, h.C, h.D, s);
  return dst;
}
template <typename T>
static void stage_out(Hier& h, int l, const T* src, void* dst, hipStream_t s) {
  launch_soa_to_aos<T, T>(src, (T*)dst, h.lv[l].n_n, h.C, h.D, s);
}

template <typename T>
static void apply_api(Hier& h, int l, int epi, const void* d_u, const void* d_f, void* d_out, hipStream_t s) {
  h.ensure_io<T>(l);
  Work<T>& W = h.work<T>();
  const T* u = stage_in<T>(h, l, d_u, W.io1[l], s);
  const T* f = d_f ? stage_in<T>(h, l, d_f, W.io2[l], s) : nullptr;
  apply<T>(h, l, epi, u, f, W.io3[l], h.C, s);
  stage_out<T>(h, l, W.io3[l], d_out, s);
}

gmt_status gmt_apply_K(gmt_hier_t H, int32_t level, const void* d_u, void* d_y, int32_t dtype, void* stream) {
  return guarded([&] {
    check_level(H, level);
    check_dtype(dtype);
    if (!d_u || !d_y) fail(GMT_E_INVAL, "null vector");
    if (d_u == d_y) fail(GMT_E_INVAL, "u and y must not alias");
    if (dtype == GMT_F64)
      apply_api<double>(H->h, level - 1, EPI_KU, d_u, nullptr, d_y, S(stream));
    else
      apply_api<float>(H->h, level - 1, EPI_KU, d_u, nullptr, d_y, S(stream));
  });
}

gmt_status gmt_residual(gmt_hier_t H, int32_t level, const void* d_f, const void* d_u, void* d_r, int32_t dtype,
                        void* stream) {
  return guarded([&] {
    check_level(H, level);
    check_dtype(dtype);
    if (!d_f || !d_u || !d_r) fail(GMT_E_INVAL, "null vector");
    if (d_r == d_u) fail(GMT_E_INVAL, "r and u must not alias");
    if (dtype == GMT_F64)
      apply_api<double>(H->h, level - 1, EPI_RESID, d_u, d_f, d_r, S(stream));
    else
      apply_api<float>(H->h, level - 1, EPI_RESID, d_u, d_f, d_r, S(stream));
  });
}

template <typename T>
static void smooth_abi(Hier& h, int l, const void* d_f, void* d_u, int nu, int sm, double p1, double p2,
                       hipStream_t s) {
  h.ensure_io<T>(l);
  Work<T>& W = h.work<T>();
  const T* f = stage_in<T>(h, l, d_f, W.io1[l], s);
  T* u = stage_in<T>(h, l, d_u, W.io2[l], s);
  T* alt = W.io3[l];
  smooth<T>(h, l, f, u, alt, W.dvec[l], nu, false, sm, p1, p2, s, sm == GMT_SMOOTH_GS && p2 != 0.0);
  stage_out<T>(h, l, u, d_u, s);
}

gmt_status gmt_smooth(gmt_hier_t H, int32_t level, const void* d_f, void* d_u, int32_t nu, int32_t smoother,
                      double p1, double p2, int32_t dtype, void* stream) {
  return guarded([&] {
    check_level(H, level);
    check_dtype(dtype);
    if (!d_f || !d_u) fail(GMT_E_INVAL, "null vector");
    if (nu < 0 || nu > 64) fail(GMT_E_INVAL, "nu out of range");
    if (smoother == GMT_SMOOTH_CHEBYSHEV && !(p2 > p1 && p1 > 0)) fail(GMT_E_INVAL, "need 0 < lo < hi");
    if (smoother != GMT_SMOOTH_CHEBYSHEV && smoother != GMT_SMOOTH_JACOBI && smoother != GMT_SMOOTH_GS)
      fail(GMT_E_INVAL, "bad smoother");
    if (smoother == GMT_SMOOTH_GS) {
      if (!(p1 > 0 && p1 < 2)) fail(GMT_E_INVAL, "Gauss-Seidel / SOR weight outside (0, 2)");
      if (p2 != 0.0 && p2 != 1.0) fail(GMT_E_INVAL, "Gauss-Seidel direction p2 must be 0 or 1");
      if (level == H->h.L) fail(GMT_E_INVAL, "the coarsest level is not smoothed");
      ensure_colours(H->h, S(stream));
    }
    if (dtype == GMT_F64)
      smooth_abi<double>(H->h, level - 1, d_f, d_u, nu, smoother, p1, p2, S(stream));
    else
      smooth_abi<float>(H->h, level - 1, d_f, d_u, nu, smoother, p1, p2, S(stream));
  });
}

template <typename T>
static void restrict_abi(Hier& h, int l, const void* d_rf, void* d_fc, hipStream_t s) {
  h.ensure_io<T>(l);
  h.ensure_io<T>(l + 1);
  Work<T>& W = h.work<T>();
  const T* rf = stage_in<T>(h, l, d_rf, W.io1[l], s);
  launch_restrict<T>(h.view<T>(l), h.view<T>(l + 1), h.Q, h.D, rf, W.io2[l + 1], s);
  stage_out<T>(h, l + 1, W.io2[l + 1], d_fc, s);
}

gmt_status gmt_restrict(gmt_hier_t H, int32_t level, const void* d_rf, void* d_fc, int32_t dtype, void* stream) {
  return guarded([&] {
    check_level(H, level);
    check_dtype(dtype);
    if (level == H->h.L) fail(GMT_E_INVAL, "no level below the coarsest");
    if (!d_rf || !d_fc) fail(GMT_E_INVAL, "null vector");
    if (dtype == GMT_F64)
      restrict_abi<double>(H->h, level - 1, d_rf, d_fc, S(stream));
    else
      restrict_abi<float>(H->h, level - 1, d_rf, d_fc, S(stream));
  });
}

template <typename T>
static void prolong_abi(Hier& h, int l, const void* d_uc, void* d_uf, hipStream_t s) {
  h.ensure_io<T>(l);
  h.ensure_io<T>(l + 1);
  Work<T>& W = h.work<T>();
  const T* uc = stage_in<T>(h, l + 1, d_uc, W.io1[l + 1], s);
  T* uf = stage_in<T>(h, l, d_uf, W.io2[l], s);
  launch_prolong_add<T>(h.view<T>(l), h.view<T>(l + 1), h.Q, h.D, uc, uf, s);
  stage_out<T>(h, l, uf, d_uf, s);
}

gmt_status gmt_prolong_add(gmt_hier_t H, int32_t level, const void* d_uc, void* d_uf, int32_t dtype, void* stream) {
  return guarded([&] {
    check_level(H, level);
    check_dtype(dtype);
    if (level == H->h.L) fail(GMT_E_INVAL, "no level below the coarsest");
    if (!d_uc || !d_uf) fail(GMT_E_INVAL, "null vector");
    if (dtype == GMT_F64)
      prolong_abi<double>(H->h, level - 1, d_uc, d_uf, S(stream));
    else
      prolong_abi<float>(H->h, level - 1, d_uc, d_uf, S(stream));
  });
}

template <typename T>
static void coarse_abi(Hier& h, const void* d_f, void* d_u, hipStream_t s) {
  const int l = h.L - 1;
  h.ensure_io<T>(l);
  Work<T>& W = h.work<T>();
  const T* f = stage_in<T>(h, l, d_f, W.io1[l], s);
  launch_coarse_solve<T>(cinv_of<T>(h), h.cn, h.D, h.C, f, W.io2[l], s);
  stage_out<T>(h, l, W.io2[l], d_u, s);
}

gmt_status gmt_coarse_solve(gmt_hier_t H, const void* d_f, void* d_u, int32_t dtype, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    check_dtype(dtype);
    if (!d_f || !d_u || d_f == d_u) fail(GMT_E_INVAL, "null or aliased vector");
    if (dtype == GMT_F64)
      coarse_abi<double>(H->h, d_f, d_u, S(stream));
    else
      coarse_abi<float>(H->h, d_f, d_u, S(stream));
  });
}

template <typename T>
static void vcycle_abi(Hier& h, const void* d_f, void* d_u, const void* const* d_e_init, const CycleCfg& cfg,
                       hipStream_t s) {
  autotune<T>(h, s);  // the launch shapes the solver uses (cached per shape class)
  h.ensure_io<T>(0);
  Work<T>& W = h.work<T>();
  const T* f = stage_in<T>(h, 0, d_f, W.io1[0], s);
  T* u = stage_in<T>(h, 0, d_u, W.io2[0], s);
  std::vector<const T*> e(h.L, nullptr);
  bool any = false;
  if (d_e_init) {
    for (int l = 1; l < h.L - 1; ++l)
      if (d_e_init[l]) {
        h.ensure_io<T>(l);
        e[l] = stage_in<T>(h, l, d_e_init[l], W.io3[l], s);
        any = true;
      }
  }
  vcycle<T>(h, f, u, false, any ? e.data() : nullptr, cfg, s);
  stage_out<T>(h, 0, u, d_u, s);
}

gmt_status gmt_vcycle(gmt_hier_t H, const void* d_f, void* d_u, const void* const* d_e_init,
                      const gmt_cycle_opts* opts, int32_t dtype, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    check_dtype(dtype);
    if (!d_f || !d_u || d_f == d_u) fail(GMT_E_INVAL, "null or aliased vector");
    Hier& h = H->h;
    const CycleCfg cfg = make_cycle(h, opts);
    if (cfg.smoother == GMT_SMOOTH_GS) ensure_colours(h, S(stream));
    if (dtype == GMT_F64)
      vcycle_abi<double>(h, d_f, d_u, d_e_init, cfg, S(stream));
    else
      vcycle_abi<float>(h, d_f, d_u, d_e_init, cfg, S(stream));
  });
}

gmt_status gmt_solve(gmt_hier_t H, const void* d_f, void* d_u, const gmt_solve_opts* opts, gmt_solve_report* report,
                     void* stream) {
  gmt_status st = GMT_OK;
  gmt_status g = guarded([&] {
    check_level(H, 1);
    if (!d_f || !d_u || d_f == d_u) fail(GMT_E_INVAL, "null or aliased vector");
    Hier& h = H->h;
    hipStream_t s = S(stream);
    const int n = h.lv[0].n_n;
    if (opts && opts->cycle.smoother == GMT_SMOOTH_GS) ensure_colours(h, s);
    double* f = scratch64(h, &h.s_f64s);
    double* u = scratch64(h, &h.s_u64s);
    const bool zero = opts && opts->zero_start;
    launch_aos_to_soa<double, double>((const double*)d_f, f, n, h.C, h.D, s);
    if (zero)
      launch_fill<double>(u, (size_t)n * h.Q, 0.0, s);
    else
      launch_aos_to_soa<double, double>((const double*)d_u, u, n, h.C, h.D, s);
    solve(h, f, u, opts, report, s, &st, zero);
    launch_soa_to_aos<double, double>(u, (double*)d_u, n, h.C, h.D, s);
    GMT_HIP(hipStreamSynchronize(s));
  });
  return g != GMT_OK ? g : st;
}

// Every buffer solve() may allocate, allocated up front (batched workers never
// allocate: the allocation callback may not be callable from their threads).
static void prepare_solve(Hier& h, int prec, const gmt_solve_opts* o, hipStream_t s) {
  const size_t tot = (size_t)h.lv[0].n_n * h.Q;
  if (o && o->cycle.smoother == GMT_SMOOTH_GS) ensure_colours(h, s);
  if (!h.pcg_flags) h.pcg_flags = h.alloc<double>(16);  // device convergence flags of the captured blocks
  scratch64(h, &h.s_f64s);
  scratch64(h, &h.s_u64s);
  scratch64(h, &h.s_r64);
  if (prec == GMT_F32) {
    if (!h.s_b32) h.s_b32 = h.alloc<float>(tot);
    if (!h.s_x32) h.s_x32 = h.alloc<float>(tot);
    scratch64(h, &h.s_usave);
    autotune<float>(h, s);
    borrow_f32_shape(h);
  } else {
    scratch64(h, &h.s_x64);
    autotune<double>(h, s);
  }
}

gmt_status gmt_solve_batch(gmt_hier_t const* hs, int32_t n, const void* const* d_f, void* const* d_u,
                           const gmt_solve_opts* opts, int32_t n_workers, gmt_solve_report* reports,
                           gmt_status* status, void* stream) {
  std::vector<gmt_status> st((size_t)std::max(n, 0), GMT_OK);
  std::vector<std::string> msg((size_t)std::max(n, 0));
  gmt_status g = guarded([&] {
    if (n < 0 || (n > 0 && (!hs || !d_f || !d_u))) fail(GMT_E_INVAL, "bad batch arguments");
    const int prec = opts ? opts->precision : GMT_F64;
    if (prec != GMT_F64 && prec != GMT_F32) fail(GMT_E_INVAL, "bad precision");
    for (int i = 0; i < n; ++i) {
      check_level(hs[i], 1);
      if (!d_f[i] || !d_u[i] || d_f[i] == d_u[i]) fail(GMT_E_INVAL, "cell %d: null or aliased vector", i);
      for (int j = 0; j < i; ++j)
        if (hs[j] == hs[i]) fail(GMT_E_INVAL, "cell %d repeats the hierarchy of cell %d", i, j);
    }
    GMT_HIP(hipStreamSynchronize(S(stream)));
    for (int i = 0; i < n; ++i) prepare_solve(hs[i]->h, prec, opts, S(stream));
    GMT_HIP(hipStreamSynchronize(S(stream)));
    // Longest-processing-time order balances the workers.  A cell's cost is its
    // unknowns times its iteration count, and the count rises steeply with the
    // share of level-1 nodes on the solid's surface (thin members): on 128^3
    // cells a share of 0.1-0.3 needs 10-25 PCG iterations, 0.4-0.46 up to 100,
    // 0.5-0.63 about 850.  exp(12 share) follows that rise closely enough to
    // start the slowest cells first.
    std::vector<double> cost(n);
    for (int i = 0; i < n; ++i) {
      const LevelData& d0 = hs[i]->h.lv[0];
      const double share = d0.n_n > 0 ? (double)d0.n_bnd / d0.n_n : 0.0;
      cost[i] = (double)d0.n_n * hs[i]->h.Q * std::exp(12.0 * share);
    }
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    int dev = 0;
    GMT_HIP(hipGetDevice(&dev));
    const int nw = std::max(1, std::min(n_workers > 0 ? n_workers : 4, std::max(n, 1)));
    std::atomic<int> next{0};
    auto worker = [&]() {
      hipStream_t ws = nullptr;
      const gmt_status ok = guarded([&] {
        GMT_HIP(hipSetDevice(dev));
        GMT_HIP(hipStreamCreateWithFlags(&ws, hipStreamNonBlocking));
      });
      for (;;) {
        const int k = next.fetch_add(1);
        if (k >= n) break;
        const int i = order[k];
        if (ok != GMT_OK) {
          st[i] = ok;
          msg[i] = g_last_error;
          continue;
        }
        gmt_status cell = GMT_OK;
        gmt_solve_report rep{};
        st[i] = guarded([&] {
          Hier& h = hs[i]->h;
          // buffers allocated from this thread (an FP64 fallback's work vectors)
          // come from hipMalloc, not from the caller's allocation callback
          struct LocalAlloc {
            Hier& h;
            explicit LocalAlloc(Hier& hh) : h(hh) { h.local_alloc = true; }
            ~LocalAlloc() { h.local_alloc = false; }
          } local(h);
          const int nn = h.lv[0].n_n;
          double* f = h.s_f64s;
          double* u = h.s_u64s;
          const bool zero = opts && opts->zero_start;
          launch_aos_to_soa<double, double>((const double*)d_f[i], f, nn, h.C, h.D, ws);
          if (zero)
            launch_fill<double>(u, (size_t)nn * h.Q, 0.0, ws);
          else
            launch_aos_to_soa<double, double>((const double*)d_u[i], u, nn, h.C, h.D, ws);
          solve(h, f, u, opts, &rep, ws, &cell, zero);
          launch_soa_to_aos<double, double>(u, (double*)d_u[i], nn, h.C, h.D, ws);
          GMT_HIP(hipStreamSynchronize(ws));
        });
        if (st[i] == GMT_OK) st[i] = cell;
        if (st[i] != GMT_OK) msg[i] = g_last_error;
        if (reports) reports[i] = rep;
      }
      if (ws) (void)hipStreamDestroy(ws);
    };
    std::vector<std::thread> pool;
    for (int w = 0; w < nw; ++w) pool.emplace_back(worker);
    for (auto& t : pool) t.join();
  });
  if (status)
    for (int i = 0; i < n; ++i) status[i] = st[i];
  if (g != GMT_OK) return g;
  for (int i = 0; i < n; ++i)
    if (st[i] != GMT_OK) {
      g_last_error = "cell " + std::to_string(i) + ": " + msg[i];
      return st[i];
    }
  return GMT_OK;
}

// caller vector (level 1, dtype) -> FP64 [Q][n] scratch
static const double* to_soa64(Hier& h, const void* src, int dtype, double** slot, hipStream_t s) {
  double* dst = scratch64(h, slot);
  if (dtype == GMT_F64)
    launch_aos_to_soa<double, double>((const double*)src, dst, h.lv[0].n_n, h.C, h.D, s);
  else
    launch_aos_to_soa<float, double>((const float*)src, dst, h.lv[0].n_n, h.C, h.D, s);
  return dst;
}

gmt_status gmt_relative_residual(gmt_hier_t H, const void* d_f, const void* d_u, int32_t dtype, double* h_rel,
                                 void* stream) {
  return guarded([&] {
    check_level(H, 1);
    check_dtype(dtype);
    if (!d_f || !d_u || !h_rel) fail(GMT_E_INVAL, "null pointer");
    Hier& h = H->h;
    hipStream_t s = S(stream);
    const double* f = to_soa64(h, d_f, dtype, &h.s_x64, s);
    const double* u = to_soa64(h, d_u, dtype, &h.s_t64, s);
    rel_residual64(h, f, u, scratch64(h, &h.s_r64), h_rel, nullptr, s);
  });
}

gmt_status gmt_homogenize(gmt_hier_t H, const void* d_u, int32_t dtype, double* h_CH, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    check_dtype(dtype);
    if (!d_u || !h_CH) fail(GMT_E_INVAL, "null pointer");
    Hier& h = H->h;
    hipStream_t s = S(stream);
    const int n = h.lv[0].n_n, C = h.C;
    const double* u = to_soa64(h, d_u, dtype, &h.s_t64, s);
    double* y = scratch64(h, &h.s_r64);
    apply<double>(h, 0, EPI_KU, u, nullptr, y, C, s);
    double* A = h.red_out + 96;
    double* B = h.red_out + 160;
    launch_gram<double, double>(h.f64, u, n, C, h.D, h.red_partial, A, s);  // A[i][j] = f_i . u_j
    launch_gram<double, double>(u, y, n, C, h.D, h.red_partial, B, s);      // B[i][j] = u_i . (K u)_j
    double Ah[36], Bh[36];
    host_dot(h, A, C * C, Ah, s);
    host_dot(h, B, C * C, Bh, s);
    const double vol = (double)h.N * h.N * h.N;
    // sum_e s_e X0^T K0 X0 = (sum_e s_e) C0 (s_e = 1 in a binary cell)
    const double ne = h.density ? h.scale_sum : (double)h.lv[0].n_e;
    for (int i = 0; i < C; ++i)
      for (int j = 0; j < C; ++j)
        h_CH[i * C + j] = (ne * h.C0[i * C + j] - Ah[i * C + j] - Ah[j * C + i] + Bh[i * C + j]) / vol;
  });
}


// ================================================================ SIMP inverse homogenization (App. F.3)

gmt_status gmt_simp_sensitivity(gmt_hier_t H, const double* d_u, const double* h_G, double* d_dJ, double* d_dC,
                                void* stream) {
  return guarded([&] {
    check_level(H, 1);
    Hier& h = H->h;
    if (!h.density) fail(GMT_E_STATE, "not a density hierarchy (gmt_build_density_hierarchy)");
    if (!d_u) fail(GMT_E_INVAL, "d_u is NULL");
    if (!d_dJ && !d_dC) fail(GMT_E_INVAL, "nothing to compute: d_dJ and d_dC are both NULL");
    if (d_dJ && !h_G) fail(GMT_E_INVAL, "d_dJ needs the weights h_G");
    hipStream_t s = S(stream);
    const LevelData& d = h.lv[0];
    const size_t n3 = (size_t)h.N * h.N * h.N;
    double* G = nullptr;
    if (h_G) {
      G = h.red_out + 200;  // c*c <= 36 values, past the reduction slots used here
      GMT_HIP(hipMemcpyAsync(G, h_G, (size_t)h.C * h.C * sizeof(double), hipMemcpyHostToDevice, s));
    }
    if (d_dJ) launch_fill<double>(d_dJ, n3, 0.0, s);
    if (d_dC) launch_fill<double>(d_dC, n3 * h.C * h.C, 0.0, s);
    launch_simp_sensitivity(d.elem_lin, d.n_e, d.node_map, h.N, h.D, h.C, d_u, h.Ke64, h.X064, d.erho, h.simp_p, G,
                            d_dJ, d_dC, s);
    GMT_HIP(hipStreamSynchronize(s));  // h_G is read by the copy above
  });
}

gmt_status gmt_simp_objective(const double* h_CH, int32_t kind, double* h_J, double* h_G) {
  return guarded([&] {
    if (!h_CH || !h_J || !h_G) fail(GMT_E_INVAL, "null pointer");
    if (kind < GMT_SIMP_YOUNG || kind > GMT_SIMP_BULK) fail(GMT_E_INVAL, "objective kind %d", kind);
    // S = C_H^-1 by Gauss-Jordan elimination with partial pivoting
    double A[6][12];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 12; ++j) A[i][j] = j < 6 ? h_CH[i * 6 + j] : (j - 6 == i ? 1.0 : 0.0);
    for (int c = 0; c < 6; ++c) {
      int piv = c;
      for (int r = c + 1; r < 6; ++r)
        if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
      if (!(std::fabs(A[piv][c]) > 0)) fail(GMT_E_SINGULAR, "C_H is singular");
      if (piv != c)
        for (int j = 0; j < 12; ++j) std::swap(A[c][j], A[piv][j]);
      const double inv = 1.0 / A[c][c];
      for (int j = 0; j < 12; ++j) A[c][j] *= inv;
      for (int r = 0; r < 6; ++r)
        if (r != c) {
          const double f = A[r][c];
          for (int j = 0; j < 12; ++j) A[r][j] -= f * A[c][j];
        }
    }
    double Sm[6][6], W[6][6] = {{0}};
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) Sm[i][j] = A[i][j + 6];
    if (kind == GMT_SIMP_YOUNG)
      for (int i = 0; i < 3; ++i) W[i][i] = 1.0 / 3.0;
    else if (kind == GMT_SIMP_SHEAR)
      for (int i = 3; i < 6; ++i) W[i][i] = 1.0 / 3.0;
    else
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) W[i][j] = 1.0;
    double J = 0.0;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) J += W[i][j] * Sm[i][j];
    *h_J = J;
    // dJ/dC = -S^T W S^T (dS = -S dC S)
    double T[6][6];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double t = 0.0;
        for (int k = 0; k < 6; ++k) t += Sm[k][i] * W[k][j];
        T[i][j] = t;
      }
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double t = 0.0;
        for (int k = 0; k < 6; ++k) t += T[i][k] * Sm[j][k];
        h_G[i * 6 + j] = -t;
      }
  });
}

gmt_status gmt_simp_filter(const double* d_rho, const double* d_dc, int32_t N, double rmin, double* d_out,
                           void* stream) {
  return guarded([&] {
    if (!d_rho || !d_dc || !d_out) fail(GMT_E_INVAL, "null pointer");
    if (N < 1 || N > 1024) fail(GMT_E_INVAL, "N = %d outside 1..1024", N);
    if (!(rmin > 1.0) || rmin > 8.0) fail(GMT_E_INVAL, "filter radius %g outside (1, 8]", rmin);
    if (d_out == d_dc || d_out == d_rho) fail(GMT_E_INVAL, "d_out must not alias the inputs");
    launch_simp_filter(d_rho, d_dc, N, rmin, 1e-3, d_out, S(stream));
  });
}

gmt_status gmt_simp_oc(const double* d_rho, const double* d_dc, size_t n, double volfrac, double move, double eta,
                       double rho_lo, double* d_rho_new, double* h_lambda, void* stream) {
  return guarded([&] {
    if (!d_rho || !d_dc || !d_rho_new) fail(GMT_E_INVAL, "null pointer");
    if (n == 0) fail(GMT_E_INVAL, "n = 0");
    if (!(volfrac > 0 && volfrac < 1) || !(move > 0) || !(eta > 0) || !(rho_lo > 0 && rho_lo < 1))
      fail(GMT_E_INVAL, "need 0 < volfrac < 1, move > 0, eta > 0, 0 < rho_lo < 1");
    if (d_rho_new == d_rho || d_rho_new == d_dc) fail(GMT_E_INVAL, "d_rho_new must not alias the inputs");
    hipStream_t s = S(stream);
    double* partial = nullptr;
    double* total = nullptr;
    GMT_HIP(hipMallocAsync((void**)&partial, (kRedBlocks + 1) * sizeof(double), s));
    total = partial + kRedBlocks;
    // bisection on the multiplier: the updated volume decreases with lam
    double lo = 0.0, hi = 1e9, lam = hi, vol = 0.0;
    const double target = volfrac * (double)n;
    for (int it = 0; it < 200; ++it) {
      lam = 0.5 * (lo + hi);
      launch_oc_eval(d_rho, d_dc, n, lam, move, eta, rho_lo, nullptr, partial, total, s);
      GMT_HIP(hipMemcpyAsync(&vol, total, sizeof(double), hipMemcpyDeviceToHost, s));
      GMT_HIP(hipStreamSynchronize(s));
      if (vol > target)
        lo = lam;
      else
        hi = lam;
      if (hi - lo <= 1e-10 * std::max(hi, 1e-30)) break;
    }
    launch_oc_eval(d_rho, d_dc, n, lam, move, eta, rho_lo, d_rho_new, partial, total, s);
    GMT_HIP(hipFreeAsync(partial, s));
    GMT_HIP(hipStreamSynchronize(s));
    if (h_lambda) *h_lambda = lam;
  });
}

// ================================================================ learned initializer

gmt_status gmt_nn_param_count(const gmt_nn_config* cfg, int32_t physics, size_t* n_params) {
  return guarded([&] {
    if (!cfg || !n_params) fail(GMT_E_INVAL, "null pointer");
    if (cfg->levels < 2 || cfg->levels > GMT_NN_MAX_LEVELS) fail(GMT_E_INVAL, "bad levels");
    if (cfg->attention != 0 && cfg->attention != 1) fail(GMT_E_INVAL, "attention must be 0 or 1");
    *n_params = nn_param_count(*cfg, physics == GMT_ELASTIC ? 18 : 3);
  });
}

gmt_status gmt_nn_setup(gmt_hier_t H, const gmt_nn_config* cfg, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    if (!cfg) fail(GMT_E_INVAL, "cfg is NULL");
    nn_setup(H->h, *cfg, S(stream));
  });
}

gmt_status gmt_nn_forward(gmt_hier_t H, const float* d_params, float* const* d_out, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    if (!d_params || !d_out) fail(GMT_E_INVAL, "null pointer");
    nn_forward(H->h, d_params, d_out, S(stream));
  });
}

gmt_status gmt_nn_backward(gmt_hier_t H, const float* const* d_gout, float* d_grad, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    if (!d_gout || !d_grad) fail(GMT_E_INVAL, "null pointer");
    nn_backward(H->h, d_gout, d_grad, S(stream));
  });
}

gmt_status gmt_nn_activation(gmt_hier_t H, int32_t level, int32_t which, float* d_out, int32_t* h_width,
                             void* stream) {
  return guarded([&] {
    check_level(H, level);
    const int w = nn_activation(H->h, level - 1, which, d_out, S(stream));
    if (h_width) *h_width = w;
  });
}

gmt_status gmt_nn_serialization(gmt_hier_t H, int32_t level, int32_t* d_order, void* stream) {
  return guarded([&] {
    check_level(H, level);
    if (!d_order) fail(GMT_E_INVAL, "null pointer");
    nn_serialization(H->h, level - 1, d_order, S(stream));
  });
}

gmt_status gmt_nn_supervised_loss(gmt_hier_t H, const float* d_pred, const float* d_target, double alpha,
                                  float* d_grad, double* h_loss, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    if (!d_pred || !d_target || !h_loss) fail(GMT_E_INVAL, "null pointer");
    if (!(alpha >= 0.0)) fail(GMT_E_INVAL, "alpha must be >= 0");
    *h_loss = nn_supervised(H->h, d_pred, d_target, alpha, d_grad, S(stream));
  });
}

gmt_status gmt_nn_time_attention(gmt_hier_t H, int32_t level, int32_t reps, double* h_ms, void* stream) {
  return guarded([&] {
    check_level(H, level);
    if (!h_ms) fail(GMT_E_INVAL, "h_ms is NULL");
    if (reps < 1 || reps > 100000) fail(GMT_E_INVAL, "reps out of range");
    *h_ms = nn_time_attention(H->h, level - 1, reps, S(stream));
  });
}

gmt_status gmt_nn_adamw(float* d_params, const float* d_grad, float* d_m, float* d_v, size_t n, double lr,
                        double beta1, double beta2, double eps, double wd, int32_t step, double grad_scale,
                        void* stream) {
  return guarded([&] {
    if (!d_params || !d_grad || !d_m || !d_v) fail(GMT_E_INVAL, "null pointer");
    if (step < 1) fail(GMT_E_INVAL, "step must be >= 1");
    nn_adamw(d_params, d_grad, d_m, d_v, n, lr, beta1, beta2, eps, wd, step, grad_scale, S(stream));
  });
}

gmt_status gmt_nn_norm2(const float* d_x, size_t n, double* h_out, void* stream) {
  return guarded([&] {
    if (!d_x || !h_out) fail(GMT_E_INVAL, "null pointer");
    *h_out = nn_norm2(nullptr, d_x, n, S(stream));
  });
}

extern "C" gmt_status gmt_nn_norm2_noalloc(const float* d_x, size_t n, double* h_out, void* stream) {
  return guarded([&] {
    if (!d_x || !h_out) fail(GMT_E_INVAL, "null pointer");
    *h_out = nn_norm2_noalloc(d_x, n, S(stream));
  });
}

gmt_status gmt_nn_ema(float* d_ema, const float* d_x, size_t n, double decay, void* stream) {
  return guarded([&] {
    if (!d_ema || !d_x) fail(GMT_E_INVAL, "null pointer");
    nn_ema(d_ema, d_x, n, decay, S(stream));
  });
}

namespace gmt {
// Loss of Sec. 4.5 after one Alg. 2 V-cycle from the predictions, and its gradient
// through the exact adjoint of the (affine) V-cycle:
//   u^1 = E_V u_hat + sum_l B_l e_hat^l + c,   E_V = I - M^-1 K   (M^-1 the V-cycle, symmetric)
//   dL/du_hat = E_V^T g = g - K M^-1 g
//   dL/de_hat^l = (I - K_l M_l^-1) R Post_{l-1}^T ... R Post_1^T g
// with Post_k^T = p(K D^-1) = D p(D^-1 K) D^-1 the transposed post-smoothing polynomial.
static void vcycle_loss(Hier& h, const float* const* d_pred, const gmt_cycle_opts* opts, double lambda,
                        float* d_u1, double* h_out, float* const* d_gpred, hipStream_t s) {
  const CycleCfg cfg = make_cycle(h, opts);
  if (cfg.smoother == GMT_SMOOTH_GS || cfg.schedule != GMT_CYCLE_V)
    fail(GMT_E_INVAL, "the loss adjoint covers the V-cycle with Chebyshev or Jacobi smoothing");
  autotune<float>(h, s);  // the launch shapes the solver uses (cached per shape class)
  h.ensure_work<float>();
  h.ensure_io<float>(0);
  Work<float>& W = h.work<float>();
  const int L = h.L, C = h.C, D = h.D, Q = h.Q;
  const int n = h.lv[0].n_n;
  const size_t tot = (size_t)n * Q;
  float* f = W.io1[0];
  launch_convert<double, float>(h.f64, f, tot, s);
  float* u = stage_in<float>(h, 0, d_pred[0], W.io2[0], s);
  std::vector<const float*> e(L, nullptr);
  bool any = false;
  for (int l = 1; l < L - 1; ++l)
    if (d_pred[l]) {
      h.ensure_io<float>(l);
      e[l] = stage_in<float>(h, l, d_pred[l], W.io3[l], s);
      any = true;
    }
  vcycle<float>(h, f, u, false, any ? e.data() : nullptr, cfg, s);
  if (d_u1) stage_out<float>(h, 0, u, d_u1, s);
  float* r = W.pr;
  apply<float>(h, 0, EPI_RESID, u, f, r, C, s);
  double* sc = h.red_out;
  double *rr = sc + 40, *ff = sc + 48, *sums = sc + 200, *add = sc + 224;
  launch_dot<float>(r, r, n, C, D, h.red_partial, rr, s);
  launch_dot<float>(f, f, n, C, D, h.red_partial, ff, s);
  launch_colsum<float>(u, n, Q, D, h.red_partial, sums, s);
  double rh[8], fh[8], sh[18];
  host_dot(h, rr, C, rh, s);
  host_dot(h, ff, C, fh, s);
  host_dot(h, sums, Q, sh, s);
  double r2 = 0, fmax = 0, pen = 0;
  for (int c = 0; c < C; ++c) {
    r2 += rh[c];
    fmax = std::max(fmax, std::sqrt(fh[c]));
  }
  for (int q = 0; q < Q; ++q) pen += sh[q] * sh[q];
  const double rn = std::sqrt(r2);
  if (h_out) {
    h_out[0] = std::log10(rn + 1e-12) + lambda * pen;
    h_out[1] = rn;
    for (int c = 0; c < C; ++c) {
      double den = std::sqrt(fh[c]);
      if (den <= 1e-12 * fmax) den = fmax;
      h_out[2 + c] = den > 0 ? std::sqrt(rh[c]) / den : 0.0;
    }
  }
  if (!d_gpred) return;
  // g = dL/du^1 = -K r / (ln10 (||r|| + 1e-12) ||r||) + 2 lambda (sum_i u^1_i) per component
  float* g = W.pz;
  apply<float>(h, 0, EPI_KU, r, nullptr, g, C, s);
  const double alpha = rn > 0 ? -1.0 / (std::log(10.0) * (rn + 1e-12) * rn) : 0.0;
  double addh[18];
  for (int q = 0; q < Q; ++q) addh[q] = 2.0 * lambda * sh[q];
  GMT_HIP(hipMemcpyAsync(add, addh, Q * sizeof(double), hipMemcpyHostToDevice, s));
  launch_scale_add_comp<float>(g, g, (float)alpha, add, n, C, D, s);
  // adjoint sweep down the levels
  float* w = g;
  for (int l = 0; l < L - 1; ++l) {
    const int nl = h.lv[l].n_n;
    const size_t tl = (size_t)nl * Q;
    float *z, *kz;
    if (l == 0) {
      z = W.pq;
      kz = W.px;
    } else {
      z = W.io2[l];
      kz = W.io3[l];
    }
    if (d_gpred[l]) {
      vcycle<float>(h, w, z, true, nullptr, cfg, s, l);
      apply<float>(h, l, EPI_KU, z, nullptr, kz, C, s);
      launch_axpby<float>(kz, w, 1.f, -1.f, tl, s);  // kz = w - K V(w)
      stage_out<float>(h, l, kz, d_gpred[l], s);
    }
    bool deeper = false;
    for (int k = l + 1; k < L - 1; ++k) deeper |= d_gpred[k] != nullptr;
    if (!deeper) break;
    // w_{l+1} = R Post_l^T w_l,  Post_l^T w = D p(D^-1 K) (D^-1 w)
    h.ensure_io<float>(l + 1);
    float* t = l == 0 ? W.pr : z;
    float* zero = kz;
    launch_copy<float>(w, t, tl, s);
    launch_mul_nodewise<float>(t, h.lv[l].dinv32, nl, C, D, 0, s);
    launch_fill<float>(zero, tl, 0.f, s);
    float* cur = t;
    float* alt = W.ualt[l];
    const double q1 = cfg.smoother == GMT_SMOOTH_JACOBI ? cfg.omega[l] : cfg.lo[l];
    smooth<float>(h, l, zero, cur, alt, W.dvec[l], cfg.nu2, false, cfg.smoother, q1, cfg.hi[l], s);
    launch_mul_nodewise<float>(cur, h.lv[l].dinv32, nl, C, D, 1, s);
    launch_restrict<float>(h.view<float>(l), h.view<float>(l + 1), Q, D, cur, W.io1[l + 1], s);
    w = W.io1[l + 1];
  }
  GMT_HIP(hipStreamSynchronize(s));
}
}  // namespace gmt

gmt_status gmt_vcycle_loss(gmt_hier_t H, const float* const* d_pred, const gmt_cycle_opts* opts, double lambda,
                           float* d_u1, double* h_out, float* const* d_gpred, void* stream) {
  return guarded([&] {
    check_level(H, 1);
    if (!d_pred || !d_pred[0]) fail(GMT_E_INVAL, "d_pred[0] (u_hat^1) is required");
    if (H->h.L < 2) fail(GMT_E_INVAL, "the learned path needs at least 2 levels");
    vcycle_loss(H->h, d_pred, opts, lambda, d_u1, h_out, d_gpred, S(stream));
  });
}
