// Internal declarations shared by the kernels and the host runtime of libgmt.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "gmt.h"

namespace gmt {

// ---------------------------------------------------------------- errors

struct Failure {
  gmt_status status;
  std::string msg;
};

[[noreturn]] void fail(gmt_status st, const char* fmt, ...);

#define GMT_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      ::gmt::fail(GMT_E_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),     \
                  __FILE__, __LINE__);                                                  \
  } while (0)

#define GMT_LAUNCH_CHECK() GMT_HIP(hipGetLastError())

// ---------------------------------------------------------------- kinds of element operator

// How the element matrices of a level are stored (Sec. 4.6 EBE form):
//   SHARED : level 1, every active voxel carries the same K_e;
//   TABLE  : level 2, K_E depends only on which of its 8 children are active,
//            so it is one of 256 precomputed Galerkin sums (index = child mask);
//   PERELEM: level >= 3, one Galerkin matrix per coarse element.
enum Kind { KIND_SHARED = 0, KIND_TABLE = 1, KIND_PERELEM = 2 };

// Symmetry classes of the isotropic voxel element.  Reflecting the unit cube
// along axis d maps corner a to a ^ (1 << d) and flips the sign of DOF d, so
// block (a, m) of K_e equals, up to the sign (-1)^(a_d + a_d2) of entry
// (d, d2), block (0, a ^ m); with the axis permutations, an entry of block
// (0, delta) depends only on (delta_d, the number of other set bits of delta)
// on the diagonal and on (delta_d, delta_d2, delta_third) off it: 14 values for
// the elastic element, 4 for the scalar one (the bit count of delta).  The host
// derives the table from K_e and checks every entry against it.
template <int D>
__host__ __device__ constexpr int kcls_index(int delta, int d, int d2) {
  if (D == 1) return ((delta & 1) + ((delta >> 1) & 1) + (delta >> 2));
  if (d == d2) {
    const int o = delta & ~(1 << d) & 7;
    return ((delta >> d) & 1) * 3 + ((o & 1) + ((o >> 1) & 1) + (o >> 2));
  }
  const int t = 3 - d - d2;
  return 6 + ((delta >> d) & 1) * 4 + ((delta >> d2) & 1) * 2 + ((delta >> t) & 1);
}
template <int D>
__host__ __device__ constexpr bool kcls_negative(int a, int d, int d2) {
  return D == 3 && ((((a >> d) & 1) + ((a >> d2) & 1)) & 1);
}

// Symmetry classes of the assembled interior stencil S (27 offsets o, D x D
// blocks).  By the same reflections and axis permutations, entry (d, d2) of
// the block of offset o is, on the diagonal, a function of (o_d != 0, the
// number of other nonzero components) and, off it, sign(o_d o_d2) times a
// function of (o_third != 0), and zero when o_d o_d2 = 0: 8 values for the
// elastic element, 4 for the scalar one (the number of nonzero components).
template <int D>
__host__ __device__ constexpr int scls_index(int j, int d, int d2) {
  const int o0 = j % 3 - 1, o1 = (j / 3) % 3 - 1, o2 = j / 9 - 1;
  const int nz = (o0 != 0) + (o1 != 0) + (o2 != 0);
  if (D == 1) return nz;
  const int od = d == 0 ? o0 : (d == 1 ? o1 : o2);
  if (d == d2) return (od != 0) * 3 + nz - (od != 0);
  const int t = 3 - d - d2;
  const int ot = t == 0 ? o0 : (t == 1 ? o1 : o2);
  return 6 + (ot != 0);
}
template <int D>
__host__ __device__ constexpr bool scls_negative(int j, int d, int d2) {
  if (D == 1 || d == d2) return false;
  const int o[3] = {j % 3 - 1, (j / 3) % 3 - 1, j / 9 - 1};
  return o[d] * o[d2] < 0;
}

// ints per row of the level-1 boundary neighbour table (27 ids + 1 pad)
constexpr int kBndStride = 28;
// uint16 neighbour slots per interior node in the staged sweep's table (27 used)
constexpr int kSlotStride = 28;
// the staged interior sweep takes the interior nodes in groups of nb = 256 or
// 512 (one workgroup each; 512 on levels with at least kStageBigFrom interior
// nodes, where the larger groups share more of their neighbourhoods) and
// copies at most stage_k(nb, fp64) distinct neighbours per thread to LDS
// (FP32: 8 per thread, 32 / 64 KB; FP64: 8 / 5 per thread, 48 / 60 KB)
constexpr int kStageBigFrom = 1 << 21;
__host__ __device__ constexpr int stage_k(int nb, bool f64) { return nb == 512 && f64 ? 5 : 8; }

template <typename T>
struct LevelView {
  int N;
  int n_n;
  const int* node_lin;
  const int* node_map;  // dense N^3 -> node id or -1
  const int* elem_map;  // dense N^3 -> element id or -1
  const uint8_t* occ8;  // per node: bit k set iff octant element k is active
  const uint8_t* cmask; // per element: bit c set iff child c is active (level >= 2)
  const T* K;           // SHARED: K_e; TABLE: 256 matrices; PERELEM: n_e matrices
  // level 1 only: nodes whose 8 voxels are all solid (assembled stencil S,
  // 27 x D x D) and the remaining boundary nodes (masked EBE)
  int n_int, n_bnd;
  int zero;  // always 0 (defeats loop-invariant hoisting of coefficient loads)
  const int* interior;
  const int* boundary;
  // level 1: chunk starts of the interior list (runs of consecutive nodes along x),
  // n_runs + 1 entries with runs[n_runs] = n_int
  int n_runs;
  const int* runs;
  // level 1: the 27 neighbour ids of boundary node t at bnd_nbrs[t * kBndStride ..]
  const int* bnd_nbrs;
  // level 1, staged interior sweep: its workgroup g takes the group of
  // interior nodes b*st_nodes .. of b = st_blk[g] and reads the distinct
  // node ids st_ids[st_off[b] .. st_off[b + 1]) (ascending) of their
  // neighbourhoods, at most the precision's cap; st_slot[t * kSlotStride + j]
  // is the position of neighbour j of interior node t among them.  The nodes
  // of the other groups (st_rest, n_st_rest ids) go through the plain interior
  // kernel.  Both counts 0: no tables.
  int st_nodes;  // nodes per group (256 or 512)
  const int* st_blk;
  int n_st_blk;
  const long long* st_off;
  const int* st_ids;
  const uint16_t* st_slot;
  const int* st_rest;
  int n_st_rest;
  const T* S;
  // level 1 of a density (SIMP) hierarchy: per node the 8 octant elements'
  // stiffness scales s = rho_min + rho^p (0 where inactive), [n_n][8]; null
  // for a binary cell (scale 1 where the occupancy bit is set)
  const T* oscale;
  const T* kcls;  // symmetry-class values of K_e (14 elastic, 4 scalar)
  const T* scls;  // symmetry-class values of S (8 elastic, 4 scalar)
  // launch shape of this level's operator sweeps (chosen by the autotuner):
  // workgroup size (64 or 256), cases per thread (1, or all c) -- levels >= 2
  // only -- and XCD-contiguous numbering
  int bs, xcd, cb;
  // levels >= 2: when `list` is set, the sweep covers only the n_list nodes
  // list[0 .. n_list) (one colour class of the Gauss-Seidel smoother)
  const int* list;
  int n_list;
};

// node-connected components of the active elements of level 1 (periodic;
// elements sharing a node are connected); parent: n_e ints of scratch
int count_components(const int* elem_lin, int n_e, const int* elem_map, int N, int* parent, int* d_count,
                     hipStream_t s);
// u[c][i][:] += omega D^-1 r[c][i][:] for the n_list nodes i of `list` (one
// colour of the Gauss-Seidel smoother)
template <typename T>
void launch_gs_update(const int* list, int n_list, int n, int D, int C, const T* dinv, const T* r, T* u, T omega,
                      hipStream_t s);

// Epilogue of a node-centric operator sweep.
// EPI_CHEB0 is the first Chebyshev step (d = rho2 D^-1 r, the previous d is not read).
enum Epi { EPI_KU = 0, EPI_RESID = 1, EPI_JACOBI = 2, EPI_CHEB = 3, EPI_CHEB0 = 4 };

template <typename T>
struct EpiArgs {
  const T* f;
  const T* dinv;  // [n_n][d]
  T* dvec;        // Chebyshev direction, written
  const T* dvec_in;  // the direction read (dvec, or the iterate when the last step started from zero)
  T* out;
  T omega;        // Jacobi weight
  T rho1, rho2;   // Chebyshev: d = rho1 d + rho2 D^-1 (f - K u)
};

// ---------------------------------------------------------------- kernel launchers (kernels.hip)

template <typename T>
void launch_apply(const LevelView<T>& L, int kind, int D, int C, int epi, const T* u,
                  const EpiArgs<T>& e, hipStream_t s);
template <typename T>
void launch_smooth_zero(int n, int D, int C, const T* f, const T* dinv, T scale, T* out, T* dvec,
                        hipStream_t s);
template <typename T>
void launch_normalize(const T* src, size_t n, const double* nrm2, T* dst, hipStream_t s);
template <typename T>
void launch_restrict(const LevelView<T>& fine, const LevelView<T>& coarse, int Q, int D, const T* rf, T* fc,
                     hipStream_t s);
template <typename T>
void launch_prolong_add(const LevelView<T>& fine, const LevelView<T>& coarse, int Q, int D, const T* uc, T* uf,
                        hipStream_t s);
template <typename T>
void launch_coarse_solve(const T* cinv, int cn, int D, int C, const T* f, T* u, hipStream_t s);
template <typename T>
void launch_fill(T* p, size_t n, T v, hipStream_t s);
template <typename Tin, typename Tout>
void launch_convert(const Tin* a, Tout* b, size_t n, hipStream_t s);
template <typename T>
void launch_copy(const T* a, T* b, size_t n, hipStream_t s);
// per-case dot products sum_{i,d} a[i][c][d] b[i][c][d] accumulated in FP64 -> out[c]
template <typename T>
void launch_dot(const T* a, const T* b, int n, int C, int D, double* partial, double* out,
                hipStream_t s);
// the same with b's column means (sums[c*D + d] / n, rounded to T) removed from b on the fly
template <typename T>
void launch_dot_centered(const T* a, const T* b, const double* sums, double inv_n, int n, int C, int D, double* partial,
                         double* out, hipStream_t s);
// Gram matrix out[c1*C + c2] = sum_{i,d} a[i][c1][d] b[i][c2][d] in FP64
template <typename Ta, typename Tb>
void launch_gram(const Ta* a, const Tb* b, int n, int C, int D, double* partial, double* out,
                 hipStream_t s);
// u += alpha[c] p ; r -= alpha[c] q  (vectors [C][n][D]); with qsums, q minus its column
// means qsums / n
template <typename T>
void launch_pcg_update(T* u, T* r, const T* p, const T* q, const double* alpha, int n, int Q, int D,
                       hipStream_t s, const double* qsums = nullptr, double inv_n = 0.0);
// dots[c] = a.b per case and sums[c*D + d] = column sums of b, in one pass
template <typename T>
void launch_dot_colsum(const T* a, const T* b, int n, int C, int D, double* partial, double* dots, double* sums,
                       hipStream_t s);
// rz[c] = r.(z - column means sums / n) and rr[c] = r.r, in one pass
template <typename T>
void launch_dot2_centered(const T* r, const T* z, const double* sums, double inv_n, int n, int C, int D,
                          double* partial, double* rz, double* rr, hipStream_t s);
// p = z + beta[c] p (with sums: z with its column means sums / n removed on the fly)
template <typename T>
void launch_pcg_direction(T* p, const T* z, const double* beta, int n, int Q, int D, hipStream_t s,
                          const double* sums = nullptr, double inv_n = 0.0);
// layout changes between the ABI's [n][C][D] and the solver's [C][n][D] (with type conversion)
template <typename Tin, typename Tout>
void launch_aos_to_soa(const Tin* a, Tout* b, int n, int C, int D, hipStream_t s);
template <typename Tin, typename Tout>
void launch_soa_to_aos(const Tin* a, Tout* b, int n, int C, int D, hipStream_t s);
// stop (nullable): device convergence flag; when set, alpha = beta = 0
void launch_pcg_alpha(const double* rz, const double* pq, double* alpha, int C, hipStream_t s,
                      const double* stop = nullptr);
void launch_pcg_beta(const double* rz_new, double* rz, double* beta, int C, hipStream_t s,
                     const double* stop = nullptr);
// flags: [0] stop, [1] iterations run, [2 + m] squared residual target of case m
void launch_pcg_check(const double* rr, int C, double* flags, hipStream_t s);
template <typename T>
void launch_gauge_shift(T* u, int n, int Q, int D, T* tmp, hipStream_t s);
// v -= column mean over nodes (projection off the rigid translations)
template <typename T>
void launch_project(T* v, int n, int Q, int D, double* partial, double* sums, hipStream_t s);
// u64 += a * (double) d
template <typename T>
void launch_accumulate(double* u, const T* d, size_t n, hipStream_t s, double a = 1.0);

// hierarchy construction kernels
void launch_voxel_elem_flags(const uint8_t* vox, size_t n, int* flags, hipStream_t s);
void launch_node_flags(const int* elem_map_or_flags, int N, int* node_flags, hipStream_t s);
void launch_coarsen_flags(const int* fine_elem_map, int Nf, int* coarse_flags, uint8_t* dense_cmask,
                          hipStream_t s);
int64_t scan_compact(const int* flags, size_t n, int* map_out, int* lin_out, int* scratch_blocks,
                     int* d_total, hipStream_t s);
size_t scan_scratch_ints(size_t n);
void launch_occ8(const int* node_lin, int n_n, const int* elem_map, int N, uint8_t* occ8,
                 hipStream_t s);
void launch_occ_flags(const uint8_t* occ8, int n, int want_full, int* flags, hipStream_t s);
void launch_run_flags(const int* interior, int n_int, const int* node_lin, int N, int* flags, hipStream_t s);
// Tables of the staged interior sweep of level 1 (see LevelView::st_*): pass 0
// writes the distinct-id count of every group of nb interior nodes to
// cnt, pass 1 (for the n_blk groups blk[], offsets per group) the ids and the
// slot table.
void launch_stage_tables(const int* interior, int n_int, const int* node_lin, const int* node_map, int N, int nb,
                         int pass, const int* blk, int n_blk, int* cnt, const long long* off, int* ids, uint16_t* slot,
                         hipStream_t s);
// out = the interior ids of the groups (nb positions each) blk[0 .. n_blk)
void launch_gather_blocks(const int* interior, int n_int, int nb, const int* blk, int n_blk, int* out, hipStream_t s);
void launch_boundary_nbrs(const int* boundary, int n_bnd, const int* node_lin, const int* node_map, int N, int* table,
                          hipStream_t s);
void launch_gather_cmask(const int* elem_lin, int n_e, const uint8_t* dense_cmask, uint8_t* cmask,
                         hipStream_t s);
void launch_elem_nodes(const int* elem_lin, int n_e, const int* node_map, int N, int* out,
                       hipStream_t s);
void launch_prol_maps(const int* node_lin, int n_n, int Nf, const int* coarse_node_map, int Nc,
                      int* idx, double* w, hipStream_t s);
// fscale (nullable, SHARED source only): per fine element scale of the shared K_e
void launch_galerkin(const int* elem_lin_c, int n_e_c, int Nc, const int* elem_map_f,
                     const uint8_t* cmask_f, const double* Ksrc, int src_kind, int D,
                     const double* Ps, const double* fscale, double* out64, float* out32, hipStream_t s);
template <typename T>
void launch_diagonal(const LevelView<T>& L, int kind, int D, T* diag, hipStream_t s);
// oscale (nullable): per node octant scales of a density hierarchy
void launch_load_vector(const int* node_lin, const uint8_t* occ8, const double* oscale, int n_n, int D, int C,
                        const double* fe, double* f, hipStream_t s);
// SIMP (App. F.3): density -> active voxels, per element rho and scale, per node octant scales
void launch_density_flags(const double* rho, size_t n, double prune, uint8_t* vox, hipStream_t s);
void launch_element_scale(const int* elem_lin, int n_e, const double* rho, double p, double rho_min, double* erho,
                          double* escale, hipStream_t s);
void launch_node_oscale(const int* node_lin, int n_n, const int* elem_map, int N, const double* escale,
                        double* o64, float* o32, hipStream_t s);
void launch_iota(int* a, int n, hipStream_t s);
// per element energies d_i^T K0 d_j (d = X0 - u_e) of a density hierarchy, scaled by
// p rho^(p-1) / N^3 into dense dC [N^3][C][C] and contracted with G into dense dJ [N^3]
void launch_simp_sensitivity(const int* elem_lin, int n_e, const int* node_map, int N, int D, int C,
                             const double* u_aos, const double* Ke, const double* X0, const double* erho, double p,
                             const double* G, double* dJ, double* dC, hipStream_t s);
void launch_simp_filter(const double* rho, const double* dc, int N, double rmin, double gamma, double* out,
                        hipStream_t s);
// sum over i of the OC update of element i for multiplier lam (and the update itself into out, if set)
void launch_oc_eval(const double* rho, const double* dc, size_t n, double lam, double move, double eta, double lo,
                    double* out, double* partial, double* total, hipStream_t s);
void launch_random(double* x, size_t n, uint64_t seed, hipStream_t s);
void launch_expand_elem_matrices(const LevelView<double>& L, int kind, int n_e, int D,
                                 const int* elem_lin, double* out, hipStream_t s);
template <typename T>
void launch_inv(const T* a, T* b, size_t n, hipStream_t s);

// ---------------------------------------------------------------- hierarchy

struct LevelData {
  int N = 0, n_e = 0, n_n = 0;
  int kind = KIND_SHARED;
  int* node_lin = nullptr;
  int* elem_lin = nullptr;
  int* node_map = nullptr;
  int* elem_map = nullptr;
  uint8_t* occ8 = nullptr;
  uint8_t* cmask = nullptr;   // per element, levels >= 2
  int* interior = nullptr;    // level 1: nodes with occupancy 255
  int* boundary = nullptr;    // level 1: the other nodes
  int n_int = 0, n_bnd = 0;
  int* runs = nullptr;        // level 1: chunk starts of `interior` (+ sentinel)
  int n_runs = 0;
  int* bnd_nbrs = nullptr;    // level 1: neighbour ids of the boundary nodes (kBndStride per node)
  int st_nodes = 0;
  long long* st_off = nullptr; // level 1: tables of the staged interior sweep (LevelView),
  int* st_ids = nullptr;       // the staged groups and the left-over nodes per precision
  uint16_t* st_slot = nullptr;
  int* st_blk32 = nullptr;
  int n_st_blk32 = 0;
  int* st_rest32 = nullptr;
  int n_st_rest32 = 0;
  int* st_blk64 = nullptr;
  int n_st_blk64 = 0;
  int* st_rest64 = nullptr;
  int n_st_rest64 = 0;
  double* oscale64 = nullptr; // level 1 of a density hierarchy: [n_n][8] octant scales
  float* oscale32 = nullptr;
  double* erho = nullptr;     // level 1 of a density hierarchy: rho and scale per element
  double* escale = nullptr;
  double* Kel64 = nullptr;    // per element, levels >= 3 (>= 2 for a density hierarchy)
  float* Kel32 = nullptr;
  double* diag64 = nullptr;   // [n_n][d]
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  double lam = 0.0;           // lambda_max(D^-1 K) estimate
  // node ids sorted by colour (x mod 2 + 2 (y mod 2) + 4 (z mod 2)), with the
  // start of every colour in col_off; level 1 also keeps the interior and
  // boundary lists split by colour and the boundary neighbour table in the
  // order of col_bnd (built on the first Gauss-Seidel use)
  int* col_nodes = nullptr;
  int col_off[9] = {0};
  int* col_int = nullptr;
  int col_int_off[9] = {0};
  int* col_bnd = nullptr;
  int col_bnd_off[9] = {0};
  int* col_bnd_nbrs = nullptr;
  int bs32 = 256, xcd32 = 1, cb32 = 0;  // launch shape of the FP32 / FP64 sweeps (autotuned;
  int bs64 = 256, xcd64 = 1, cb64 = 0;  // cb 0 = all cases per thread)
  bool tuned32 = false, tuned64 = false;
};

template <typename T>
struct Work {
  bool ready = false;
  std::vector<T*> f, u, ualt, dvec, r;  // per level (f[0], u[0] unused: caller owns them)
  std::vector<T*> io1, io2, io3;        // per level staging for the ABI layout changes
  T *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr, *px = nullptr;  // PCG vectors
};

struct Hier {
  gmt_params p{};
  int N = 0, L = 0, C = 0, D = 0, Q = 0;
  std::vector<LevelData> lv;
  double Ke[576] = {0};
  double fe[576] = {0};  // K_e X0, (8d) x c row-major
  double C0[36] = {0};   // X0^T K_e X0 (= base tensor)
  double X0[576] = {0};  // nodal affine fields, (8d) x c row-major
  double* X064 = nullptr;
  // density (SIMP) hierarchy: K_e of element e is s_e K0, s_e = rho_min + rho_e^p
  bool density = false;
  double simp_p = 3.0, simp_rho_min = 1e-3, simp_prune = 0.0;
  double scale_sum = 0.0;  // sum_e s_e (the n_e of a binary cell)
  double fe_norm = 0;    // ||f_e||_F, the scale of a nonzero load
  double* Ke64 = nullptr;
  float* Ke32 = nullptr;
  double* S64 = nullptr;  // assembled interior stencil, 27 x D x D
  float* S32 = nullptr;
  double* kcls64 = nullptr;  // symmetry-class values of K_e
  float* kcls32 = nullptr;
  double* scls64 = nullptr;  // symmetry-class values of S
  float* scls32 = nullptr;
  double* fe64 = nullptr;
  double* table64 = nullptr;
  float* table32 = nullptr;
  double* Ps = nullptr;  // 8 children x 8 x 8 local prolongation weights
  double* cinv64 = nullptr;
  float* cinv32 = nullptr;
  int cn = 0;
  double* f64 = nullptr;      // load vector (level 1)
  double* red_partial = nullptr;
  double* red_out = nullptr;  // small device scratch for reductions / PCG scalars
  double* pcg_flags = nullptr;  // device convergence flags of the captured PCG blocks (16 values)
  double* pcg_status = nullptr; // pinned host copies of [stop, iterations, ||r_m||^2 x 8], two slots
  hipEvent_t pcg_ev[2] = {nullptr, nullptr};  // completion of the block whose status is in each slot
  double* gauge_tmp64 = nullptr;
  float* gauge_tmp32 = nullptr;
  Work<float> w32;
  Work<double> w64;
  // FP64 / FP32 level-1 scratch vectors of the solve and query entry points
  double *s_r64 = nullptr, *s_t64 = nullptr, *s_x64 = nullptr, *s_f64s = nullptr, *s_u64s = nullptr;
  double* s_usave = nullptr;  // the iterate before an FP32 refinement step (exact undo)
  float *s_b32 = nullptr, *s_x32 = nullptr;
  std::vector<void*> owned;      // from the caller's allocation callback
  std::vector<void*> owned_hip;  // from hipMalloc (no callback, or local_alloc)
  bool local_alloc = false;      // allocate with hipMalloc even when a callback is set
  void* nn = nullptr;  // learned-initializer state (nn.hip)
  // captured blocks of inner PCG iterations (1 and 4 iterations), per precision;
  // valid while `key` (cycle parameters and iterate buffer) is unchanged
  struct PcgGraphs {
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    std::vector<double> key;
  };
  PcgGraphs g32, g64, gmx;  // FP32, FP64, FP64 Krylov with the FP32 V-cycle
  hipStream_t cap = nullptr;  // non-blocking stream used only to record the captures
  void release_graphs();

  void* raw_alloc(size_t bytes);
  void release(void* ptr);  // frees one buffer obtained from raw_alloc
  template <typename T>
  T* alloc(size_t n) {
    return static_cast<T*>(raw_alloc(n * sizeof(T) + 16));
  }
  void release_all();

  template <typename T>
  LevelView<T> view(int l) const;
  template <typename T>
  Work<T>& work();
  template <typename T>
  void ensure_work();
  template <typename T>
  void ensure_io(int l);  // staging buffers io1/io2/io3 of level l
};

constexpr int kRedBlocks = 1024;

// learned initializer (nn.hip)
void nn_setup(Hier& h, const gmt_nn_config& cfg, hipStream_t s);
void nn_release(Hier& h);
size_t nn_param_count(const gmt_nn_config& cfg, int q);
void nn_forward(Hier& h, const float* params, float* const* out, hipStream_t s);
void nn_backward(Hier& h, const float* const* gout, float* grad, hipStream_t s);
void nn_adamw(float* p, const float* g, float* m, float* v, size_t n, double lr, double b1, double b2, double eps,
              double wd, int step, double gscale, hipStream_t s);
double nn_norm2(Hier* h, const float* x, size_t n, hipStream_t s);
// the same norm with partial sums in a fixed device array (no allocation)
double nn_norm2_noalloc(const float* x, size_t n, hipStream_t s);
size_t nn_norm2_noalloc_max();
int nn_activation(Hier& h, int l, int which, float* out, hipStream_t s);
void nn_serialization(Hier& h, int l, int* out, hipStream_t s);
double nn_time_attention(Hier& h, int l, int reps, hipStream_t s);
double nn_supervised(Hier& h, const float* p, const float* t, double alpha, float* grad, hipStream_t s);
void nn_ema(float* e, const float* x, size_t n, double decay, hipStream_t s);

// attention block of the learned initializer (attention.hip): Morton serialization
// of a level's nodes (order[rank] = node, inv[node] = rank, ser_lin[rank] = linear
// index), the window of a level, and windowed Ra-RoPE attention over tensors kept
// in serialization order
int attention_window(int level);
void attention_serialize(const int* node_map, int N, int n, int view, int* order, int* inv, int* ser_lin,
                         hipStream_t s);
void attention_forward(int n, int W, int C, int N, const int* ser_lin, const uint16_t* q, const uint16_t* k,
                       const uint16_t* v, float* o32, uint16_t* o16, float* lse, hipStream_t s);
void attention_backward(int n, int W, int C, int N, const int* ser_lin, const uint16_t* q, const uint16_t* k,
                        const uint16_t* v, const float* o32, const float* lse, const float* go, float* dq, float* dk,
                        float* dv, hipStream_t s);
// column sums over nodes of a [C][n][D] vector -> sums[Q] (FP64)
template <typename T>
void launch_colsum(const T* v, int n, int Q, int D, double* partial, double* sums, hipStream_t s);
// y = alpha * x + beta * y  (elementwise)
template <typename T>
void launch_axpby(T* y, const T* x, T alpha, T beta, size_t n, hipStream_t s);
// y[(c*n+i)*D+d] = alpha * x[...] + add[c*D+d]   (per-component constant, FP64 add)
template <typename T>
void launch_scale_add_comp(T* y, const T* x, T alpha, const double* add, int n, int C, int D, hipStream_t s);
// v[(c*n+i)*D+d] *= w[i*D+d] (mode 0) or /= w[i*D+d] (mode 1)
template <typename T>
void launch_mul_nodewise(T* v, const T* w, int n, int C, int D, int divide, hipStream_t s);  // fixed grid of the two-stage reductions (deterministic order)

}  // namespace gmt
