// gfx950 kernels of libgmt: node-centric EBE operator sweeps, transfers,
// reductions and the hierarchy-construction passes.
//
// Node-centric EBE (Sec. 4.6): y_i = sum over the (up to) 8 active elements e
// around node i of the 3 (elastic) / 1 (thermal) rows of K_e belonging to
// i's local corner, times the element vector u_e.  Summed over all nodes this
// performs exactly the element products of sum_e A_e^T K_e A_e u, without
// atomics, so every result is deterministic.
//
// Solver vectors are stored case-major: value (case c, DOF d) of node i lives
// at v[(c*n + i)*D + d].  The 64 lanes of a wave that gather one neighbour's
// D DOFs of one case read one contiguous run of 64*D words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>

#include "common.h"

namespace gmt {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int wrapm(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

// Workgroups of a launch are handed to the 8 XCDs round-robin (workgroup b runs
// on XCD b mod 8).  This renumbering gives XCD k the k-th contiguous share of
// the index range instead, so that nodes that are neighbours on the grid (and
// therefore read the same vector entries) are processed under one XCD's L2.
// It is a bijection of [0, gridDim.x).
__device__ __forceinline__ int xcd_block() {
  const int B = (int)gridDim.x, b = (int)blockIdx.x;
  const int x = b & 7, q = B >> 3, r = B & 7;
  return x * q + min(x, r) + (b >> 3);
}

__device__ __forceinline__ int block_index(int xcd) { return xcd ? xcd_block() : (int)blockIdx.x; }

// Read-only operator coefficients are read through the constant address space:
// together with a wave-uniform address this gives scalar loads even inside loops
// that store to other buffers.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// index of (case c, node i, DOF d) in a case-major solver vector of n nodes
__device__ __forceinline__ size_t vix(int c, size_t n, size_t i, int D, int d) { return ((size_t)c * n + i) * D + d; }

// ---------------------------------------------------------------- operator sweeps

// Epilogue of one (case, DOF) value at idx = (c*n + i)*D + d, with D^-1 of the
// node already loaded (it is shared by the C cases).
template <typename T, int EPI>
__device__ __forceinline__ void epilogue_d(const EpiArgs<T>& e, size_t idx, T acc, T uself, T dinv) {
  if constexpr (EPI == EPI_KU) {
    e.out[idx] = acc;
  } else if constexpr (EPI == EPI_RESID) {
    e.out[idx] = e.f[idx] - acc;
  } else if constexpr (EPI == EPI_JACOBI) {
    e.out[idx] = uself + e.omega * dinv * (e.f[idx] - acc);
  } else if constexpr (EPI == EPI_CHEB) {
    const T dn = e.rho1 * e.dvec_in[idx] + e.rho2 * dinv * (e.f[idx] - acc);
    e.dvec[idx] = dn;
    e.out[idx] = uself + dn;
  } else {  // EPI_CHEB0
    const T dn = e.rho2 * dinv * (e.f[idx] - acc);
    e.dvec[idx] = dn;
    e.out[idx] = uself + dn;
  }
}

template <int EPI>
constexpr bool needs_dinv() {
  return EPI == EPI_JACOBI || EPI == EPI_CHEB || EPI == EPI_CHEB0;
}

// Epilogue of node i for the CC cases c0, c0 + 1, .. and the D DOFs, with the
// accumulated K.u in acc[c*D + q].  Every input (f, the Chebyshev direction,
// D^-1 and the node's own values, each from registers when the caller has
// them, else from memory) is loaded before the first store: the outputs may
// alias the inputs as far as the compiler can tell, so a load placed after a
// store could not be moved above it, and each value would cost its own
// round trip.  The arithmetic is that of epilogue_d.
template <typename T, int EPI, int CC, int D>
__device__ __forceinline__ void epilogue_node(const EpiArgs<T>& e, const T* __restrict__ u, size_t n, size_t i, int c0,
                                              const T* acc, const T* uself, const T* dv, const T* fpre = nullptr,
                                              const T* dpre = nullptr) {
  T fv[CC][D], dd[CC][D], us[CC][D], di[D];
#pragma unroll
  for (int q = 0; q < D; ++q) di[q] = needs_dinv<EPI>() ? (dv ? dv[q] : e.dinv[i * D + q]) : T(0);
#pragma unroll
  for (int c = 0; c < CC; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const size_t idx = vix(c0 + c, n, i, D, q);
      fv[c][q] = EPI != EPI_KU ? (fpre ? fpre[c * D + q] : e.f[idx]) : T(0);
      dd[c][q] = EPI == EPI_CHEB ? (dpre ? dpre[c * D + q] : e.dvec_in[idx]) : T(0);
      us[c][q] = needs_dinv<EPI>() ? (uself ? uself[c * D + q] : u[idx]) : T(0);
    }
  // results first, then each output array's D values of a case as one run of
  // stores (interleaving stores to the two possibly aliasing arrays would keep
  // them from merging into one wide store)
  T o[CC][D], dn[CC][D];
#pragma unroll
  for (int c = 0; c < CC; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const T a = acc[c * D + q];
      dn[c][q] = T(0);
      if constexpr (EPI == EPI_KU) {
        o[c][q] = a;
      } else if constexpr (EPI == EPI_RESID) {
        o[c][q] = fv[c][q] - a;
      } else if constexpr (EPI == EPI_JACOBI) {
        o[c][q] = us[c][q] + e.omega * di[q] * (fv[c][q] - a);
      } else if constexpr (EPI == EPI_CHEB) {
        dn[c][q] = e.rho1 * dd[c][q] + e.rho2 * di[q] * (fv[c][q] - a);
        o[c][q] = us[c][q] + dn[c][q];
      } else {  // EPI_CHEB0
        dn[c][q] = e.rho2 * di[q] * (fv[c][q] - a);
        o[c][q] = us[c][q] + dn[c][q];
      }
    }
#pragma unroll
  for (int c = 0; c < CC; ++c) {
    if constexpr (EPI == EPI_CHEB || EPI == EPI_CHEB0) {
#pragma unroll
      for (int q = 0; q < D; ++q) e.dvec[vix(c0 + c, n, i, D, q)] = dn[c][q];
    }
#pragma unroll
    for (int q = 0; q < D; ++q) e.out[vix(c0 + c, n, i, D, q)] = o[c][q];
  }
}

// Structural zeros of the assembled interior stencil of the isotropic voxel
// element: block (offset j, row d, column d2) vanishes unless d == d2 or the
// offset has nonzero components along both d and d2 (elastic); for the
// scalar problem the six face neighbours vanish.  Checked on the host.
template <int D>
__host__ __device__ constexpr bool stencil_nonzero(int j, int d, int d2) {
  const int o[3] = {j % 3 - 1, (j / 3) % 3 - 1, j / 9 - 1};
  if constexpr (D == 1) {
    const int nz = (o[0] != 0) + (o[1] != 0) + (o[2] != 0);
    return nz != 1;
  } else {
    return d == d2 || (o[d] != 0 && o[d2] != 0);
  }
}

// The symmetry-class values of the interior stencil, wave-uniform (scalar
// registers), and the signed coefficient of block entry (j, q, q2).
template <typename T, int D>
struct StencilClasses {
  static constexpr int NS = D == 1 ? 4 : 8;
  T v[NS];
  __device__ __forceinline__ explicit StencilClasses(const T* p) {
    const cptr<T> c = as_const(p);
#pragma unroll
    for (int k = 0; k < NS; ++k) v[k] = c[k];
  }
  __device__ __forceinline__ T operator()(int j, int q, int q2) const {
    const T a = v[scls_index<D>(j, q, q2)];
    return scls_negative<D>(j, q, q2) ? -a : a;
  }
};

// 27 neighbour ids of node (x,y,z) from the dense node map; runs along x of an
// all-active row are consecutive ids, so an interior node needs 9 lookups.
template <bool INTERIOR>
__device__ __forceinline__ void neighbour_ids(const int* __restrict__ map, int N, int x, int y, int z, int nb[27]) {
  const int xs[3] = {wrapm(x - 1, N), x, wrapm(x + 1, N)};
  const int ys[3] = {wrapm(y - 1, N), y, wrapm(y + 1, N)};
  const int zs[3] = {wrapm(z - 1, N), z, wrapm(z + 1, N)};
  const bool run = INTERIOR && x > 0 && x < N - 1;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int row = N * (ys[r % 3] + N * zs[r / 3]);
    if (run) {
      const int b = map[xs[0] + row];
      nb[3 * r + 0] = b;
      nb[3 * r + 1] = b + 1;
      nb[3 * r + 2] = b + 2;
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) nb[3 * r + a] = map[xs[a] + row];
    }
  }
}

// Level 1, interior nodes (all 8 surrounding voxels solid): the assembled
// 27-point stencil S of the shared K_e, wave-uniform coefficients.
// PRE: all 27 x D values of a case are loaded before the first FMA, which
// keeps 27 gathers per wave in flight at the cost of registers (occupancy).
template <typename T, int D, int EPI, int PRE = 0>
__global__ __launch_bounds__(kBlock) void k_apply_interior(LevelView<T> L, int C, const T* __restrict__ u, EpiArgs<T> e) {
  const int t = block_index(L.xcd) * kBlock + threadIdx.x;
  if (t >= L.n_int) return;
  const int i = L.interior[t];
  const int N = L.N;
  const size_t n = (size_t)L.n_n;
  const int lin = L.node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  int nb[27];
  neighbour_ids<true>(L.node_map, N, x, y, z, nb);
  T dv[D];
#pragma unroll
  for (int q = 0; q < D; ++q) dv[q] = needs_dinv<EPI>() ? e.dinv[(size_t)i * D + q] : T(0);
  const StencilClasses<T, D> S(L.scls);
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    T acc[D];
#pragma unroll
    for (int q = 0; q < D; ++q) acc[q] = T(0);
    T uself[D];
    T w[PRE ? 27 : 1][D];
    if constexpr (PRE) {
#pragma unroll
      for (int j = 0; j < 27; ++j)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) w[j][q2] = u[vix(c, n, nb[j], D, q2)];
      __builtin_amdgcn_sched_barrier(0);  // keep the scheduler from sinking the loads into the FMA chain
    }
#pragma unroll
    for (int j = 0; j < 27; ++j) {
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) {
        const T v = PRE ? w[PRE ? j : 0][q2] : u[vix(c, n, nb[j], D, q2)];
        if (j == 13) uself[q2] = v;
#pragma unroll
        for (int q = 0; q < D; ++q)
          if (stencil_nonzero<D>(j, q, q2)) acc[q] = fma(S(j, q, q2), v, acc[q]);
      }
    }
    epilogue_node<T, EPI, 1, D>(e, u, n, i, c, acc, uself, dv);
  }
}


// Level 1, interior nodes, neighbourhoods staged in LDS.  Workgroup g takes
// the NB interior nodes of group b = st_blk[g] and, per case, first copies the
// distinct vector entries that their 27-point stencils read (one gather per
// distinct node, about 4 per interior node on a lattice cell instead of 27)
// into LDS, then applies the stencil from there through the node's 27 slots.
// The plain kernel's per-node gathers keep the vector memory data path busy
// (each wide gather occupies it for ~30 cycles); here most reads go to LDS.
// A workgroup stages at most kStageK distinct nodes per thread; the groups
// with more are left to the plain kernel (st_rest).
template <typename T, int D, int EPI, int NB>
__global__ __launch_bounds__(NB) void k_apply_interior_stage(LevelView<T> L, int C, const T* __restrict__ u,
                                                             EpiArgs<T> e) {
  constexpr int kStageNodes = NB;
  constexpr int kStageK = stage_k(NB, sizeof(T) == 8);
  // an FP32 node's 3 values at a 16-byte stride: one 128-bit LDS read each
  constexpr int DP = (D == 3 && sizeof(T) == 4) ? 4 : D;
  __shared__ __align__(16) T stg[kStageK * kStageNodes * DP];
  const int g = block_index(L.xcd);
  const int b = L.st_blk[g];
  const int t = b * kStageNodes + (int)threadIdx.x;
  const bool valid = t < L.n_int;
  const size_t n = (size_t)L.n_n;
  const long long o0 = L.st_off[b];
  const int U = (int)(L.st_off[b + 1] - o0);
  int sid[kStageK];
#pragma unroll
  for (int k = 0; k < kStageK; ++k) {
    const int p = (int)threadIdx.x + k * kStageNodes;
    sid[k] = p < U ? L.st_ids[o0 + p] : -1;
  }
  // the node's 27 slots, two per 32-bit word
  unsigned sw[kSlotStride / 2];
  const int i = valid ? L.interior[t] : 0;
  if (valid) {
    const uint2* row = reinterpret_cast<const uint2*>(L.st_slot + (size_t)t * kSlotStride);
#pragma unroll
    for (int k = 0; k < kSlotStride / 4; ++k) {
      const uint2 v = row[k];
      sw[2 * k] = v.x;
      sw[2 * k + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kSlotStride / 2; ++k) sw[k] = 0;
  }
  T dv[D];
#pragma unroll
  for (int q = 0; q < D; ++q) dv[q] = needs_dinv<EPI>() && valid ? e.dinv[(size_t)i * D + q] : T(0);
  const StencilClasses<T, D> S(L.scls);
  // One case ahead: the staged values, f and the Chebyshev direction of case
  // c + 1 are loaded while case c is computed from LDS, so that each case
  // waits for one round trip to memory at most.
  T w[kStageK][D], fn[D], dn[D];
  auto load_case = [&](int c) {
    // chunks past the workgroup's count are skipped as a whole (U is uniform);
    // inside the last chunk, lanes past it load node 0's values unconditionally,
    // so that the D loads of a node merge into one
#pragma unroll
    for (int k = 0; k < kStageK; ++k)
      if (k * kStageNodes < U) {
        const size_t id = sid[k] >= 0 ? (size_t)sid[k] : 0;
#pragma unroll
        for (int q = 0; q < D; ++q) w[k][q] = u[vix(c, n, id, D, q)];
      }
#pragma unroll
    for (int q = 0; q < D; ++q) {  // (threads without a node read node 0's: i = 0)
      const size_t idx = vix(c, n, i, D, q);
      fn[q] = EPI != EPI_KU ? e.f[idx] : T(0);
      dn[q] = EPI == EPI_CHEB ? e.dvec_in[idx] : T(0);
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int k = 0; k < kStageK; ++k)
      if (k * kStageNodes < U && sid[k] >= 0) {
        T* dst = stg + ((int)threadIdx.x + k * kStageNodes) * DP;
        if constexpr (DP == 4) {
          *reinterpret_cast<float4*>(dst) = make_float4(w[k][0], w[k][1], w[k][2], 0.0f);
        } else {
#pragma unroll
          for (int q = 0; q < D; ++q) dst[q] = w[k][q];
        }
      }
  };
  load_case(0);
  store_stage();
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    T fc[D], dc[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
      fc[q] = fn[q];
      dc[q] = dn[q];
    }
    if (c + 1 < C) load_case(c + 1);
    if (valid) {
      T acc[D], uself[D];
#pragma unroll
      for (int q = 0; q < D; ++q) acc[q] = T(0);
#pragma unroll
      for (int j = 0; j < 27; ++j) {
        const int slot = (int)((sw[j >> 1] >> (16 * (j & 1))) & 0xffffu);
        T vv[D];
        if constexpr (DP == 4) {
          const float4 f4 = *reinterpret_cast<const float4*>(stg + slot * 4);
          vv[0] = f4.x;
          vv[1] = f4.y;
          vv[2] = f4.z;
        } else {
#pragma unroll
          for (int q2 = 0; q2 < D; ++q2) vv[q2] = stg[slot * D + q2];
        }
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) {
          const T v = vv[q2];
          if (j == 13) uself[q2] = v;
#pragma unroll
          for (int q = 0; q < D; ++q)
            if (stencil_nonzero<D>(j, q, q2)) acc[q] = fma(S(j, q, q2), v, acc[q]);
        }
      }
      epilogue_node<T, EPI, 1, D>(e, u, n, i, c, acc, uself, dv, fc, dc);
    }
    if (c + 1 < C) {
      __syncthreads();  // every read of case c's stage is done
      store_stage();
      __syncthreads();
    }
  }
}

// Level 1, interior nodes in runs: a thread takes up to kRun consecutive
// interior nodes of one x-row (consecutive ids).  Their 27-point stencils
// overlap, so each of the 9 neighbour rows is read once as kRun + 2 columns
// (instead of 3 columns per node) and the 9 row lookups are shared by the run.
constexpr int kRun = 4;
template <typename T, int D, int EPI>
__global__ __launch_bounds__(kBlock) void k_apply_interior_run(LevelView<T> L, int C, const T* __restrict__ u,
                                                               EpiArgs<T> e) {
  const int k = block_index(L.xcd) * kBlock + threadIdx.x;
  if (k >= L.n_runs) return;
  const int t0 = L.runs[k];
  const int len = L.runs[k + 1] - t0;  // 1 .. kRun
  const int i0 = L.interior[t0];       // the run's ids are i0 .. i0 + len - 1
  const int N = L.N;
  const size_t n = (size_t)L.n_n;
  const int lin = L.node_lin[i0];
  const int x0 = lin % N, y = (lin / N) % N, z = lin / (N * N);
  const int ys[3] = {wrapm(y - 1, N), y, wrapm(y + 1, N)};
  const int zs[3] = {wrapm(z - 1, N), z, wrapm(z + 1, N)};
  // columns x0 - 1 .. x0 + len of each row are active; without a periodic wrap
  // inside that span their ids are consecutive
  const bool fast = x0 > 0 && x0 + len < N;
  int rb[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const int row = N * (ys[r % 3] + N * zs[r / 3]);
    rb[r] = fast ? L.node_map[x0 - 1 + row] : row;
  }
  T dv[kRun][D];
#pragma unroll
  for (int m = 0; m < kRun; ++m)
#pragma unroll
    for (int q = 0; q < D; ++q)
      dv[m][q] = (needs_dinv<EPI>() && m < len) ? e.dinv[(size_t)(i0 + m) * D + q] : T(0);
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    // L.zero is 0 at run time: the coefficient address stays wave-uniform (scalar
    // loads) but depends on c, so the loads are not hoisted out of the case loop
    const cptr<T> S = as_const(L.S + (c & L.zero));
    T acc[kRun][D], uself[kRun][D];
#pragma unroll
    for (int m = 0; m < kRun; ++m)
#pragma unroll
      for (int q = 0; q < D; ++q) acc[m][q] = uself[m][q] = T(0);
#pragma unroll
    for (int r = 0; r < 9; ++r) {
#pragma unroll
      for (int col = 0; col < kRun + 2; ++col) {
        if (col > len + 1) break;
        const int id = fast ? rb[r] + col : L.node_map[wrapm(x0 - 1 + col, N) + rb[r]];
        T v[D];
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) v[q2] = u[vix(c, n, id, D, q2)];
#pragma unroll
        for (int m = 0; m < kRun; ++m) {
          const int jx = col - m;  // this column's offset + 1 from node m
          if (jx < 0 || jx > 2) continue;
          const int j = 9 * (r / 3) + 3 * (r % 3) + jx;
          if (r == 4 && jx == 1) {
#pragma unroll
            for (int q = 0; q < D; ++q) uself[m][q] = v[q];
          }
#pragma unroll
          for (int q = 0; q < D; ++q)
#pragma unroll
            for (int q2 = 0; q2 < D; ++q2)
              if (stencil_nonzero<D>(j, q, q2)) acc[m][q] = fma(S[(j * D + q) * D + q2], v[q2], acc[m][q]);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < kRun; ++m)
      if (m < len) {
#pragma unroll
        for (int q = 0; q < D; ++q)
          epilogue_d<T, EPI>(e, vix(c, n, i0 + m, D, q), acc[m][q], uself[m][q], dv[m][q]);
      }
  }
}

// chunk starts of the interior list: t begins a run unless it continues the
// previous interior node along x (next id, next linear index) and x is not a
// multiple of kRun
// Level 1: the 27 neighbour ids (-1: inactive) of every boundary node, in
// rows of kBndStride ints (16-byte aligned), so that a sweep reads them with
// a few wide loads instead of 27 dense-map lookups.
__global__ void k_boundary_nbrs(const int* __restrict__ boundary, int n_bnd, const int* __restrict__ node_lin,
                                const int* __restrict__ node_map, int N, int* __restrict__ table) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n_bnd) return;
  const int lin = node_lin[boundary[t]];
  int nb[27];
  neighbour_ids<false>(node_map, N, lin % N, (lin / N) % N, lin / (N * N), nb);
  int* row = table + (size_t)t * kBndStride;
#pragma unroll
  for (int j = 0; j < 27; ++j) row[j] = nb[j];
  row[27] = -1;
}

__global__ void k_run_flags(const int* __restrict__ interior, int n_int, const int* __restrict__ node_lin, int N,
                            int* __restrict__ flags) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n_int) return;
  const int i = interior[t];
  const int lin = node_lin[i];
  int f = 1;
  if (t > 0) {
    const int ip = interior[t - 1];
    f = !(ip == i - 1 && node_lin[ip] == lin - 1 && (lin % N) % kRun != 0);
  }
  flags[t] = f;
}

// The same two level-1 operators with the loop order turned round: each
// neighbour (interior) or element corner (boundary) is loaded for all C cases
// at once and its coefficient block is applied to every case, so a node's
// neighbourhood is read in one pass instead of C passes (shorter reuse
// distance for the neighbouring waves' gathers, one scalar load per
// coefficient per wave).  The autotuner picks between the two orders.
template <typename T, int D, int C, int EPI>
__global__ __launch_bounds__(kBlock) void k_apply_interior_nc(LevelView<T> L, const T* __restrict__ u, EpiArgs<T> e) {
  const int t = block_index(L.xcd) * kBlock + threadIdx.x;
  if (t >= L.n_int) return;
  const int i = L.interior[t];
  const int N = L.N;
  const size_t n = (size_t)L.n_n;
  const int lin = L.node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  int nb[27];
  neighbour_ids<true>(L.node_map, N, x, y, z, nb);
  const StencilClasses<T, D> S(L.scls);
  T acc[C][D], uself[C][D];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) acc[c][q] = T(0);
#pragma unroll
  for (int j = 0; j < 27; ++j) {
    T v[C][D];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) v[c][q2] = u[vix(c, n, nb[j], D, q2)];
    if (j == 13) {
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int q = 0; q < D; ++q) uself[c][q] = v[c][q];
    }
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2)
        if (stencil_nonzero<D>(j, q, q2)) {
          const T sc = S(j, q, q2);
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c][q] = fma(sc, v[c][q2], acc[c][q]);
        }
  }
  epilogue_node<T, EPI, C, D>(e, u, n, i, 0, &acc[0][0], &uself[0][0], nullptr);
}

template <typename T, int D, int C, int EPI>
__global__ __launch_bounds__(kBlock) void k_apply_boundary_nc(LevelView<T> L, const T* __restrict__ u, EpiArgs<T> e) {
  const int t = block_index(L.xcd) * kBlock + threadIdx.x;
  if (t >= L.n_bnd) return;
  const int i = L.boundary[t];
  const int N = L.N;
  const size_t n = (size_t)L.n_n;
  const int lin = L.node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  int nb[27];
  neighbour_ids<false>(L.node_map, N, x, y, z, nb);
  const unsigned occ = L.occ8[i];
  constexpr int M = 8 * D;
  const cptr<T> K = as_const(L.K);
  T acc[C][D];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) acc[c][q] = T(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (occ & (1u << k)) {
      const int a = 7 - k;
      const int ak = k & 1, bk = (k >> 1) & 1, ck = (k >> 2) & 1;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        // corners of an active element are active: nb >= 0
        const int id = nb[(ak + (m & 1)) + 3 * (bk + ((m >> 1) & 1)) + 9 * (ck + ((m >> 2) & 1))];
        T v[C][D];
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int q2 = 0; q2 < D; ++q2) v[c][q2] = u[vix(c, n, id, D, q2)];
#pragma unroll
        for (int q = 0; q < D; ++q)
#pragma unroll
          for (int q2 = 0; q2 < D; ++q2) {
            const T kc = K[(a * D + q) * M + m * D + q2];
#pragma unroll
            for (int c = 0; c < C; ++c) acc[c][q] = fma(kc, v[c][q2], acc[c][q]);
          }
      }
    }
  }
  epilogue_node<T, EPI, C, D>(e, u, n, i, 0, &acc[0][0], nullptr, nullptr);
}

// Level 1, boundary nodes, as a masked stencil: the 3x3 coefficient block of
// neighbour j is the sum, over the active octant elements that contain both
// the node and j, of the matching block of K_e (wave-uniform scalar loads
// times a per-lane 0/1 occupancy factor).  Each neighbour is then loaded once
// for all C cases, as in the interior kernel, and no lane diverges on the
// occupancy pattern.  The neighbour loop is not unrolled (uniform trip count),
// which keeps the live set to one neighbour's values and one coefficient block.
template <typename T, int D, int C, int EPI>
__global__ __launch_bounds__(kBlock) void k_apply_boundary_st(LevelView<T> L, const T* __restrict__ u, EpiArgs<T> e) {
  const int t = block_index(L.xcd) * kBlock + threadIdx.x;
  if (t >= L.n_bnd) return;
  const int i = L.boundary[t];
  const int N = L.N;
  const size_t n = (size_t)L.n_n;
  const int lin = L.node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  const unsigned occ = L.occ8[i];
  constexpr int M = 8 * D;
  const cptr<T> K = as_const(L.K);
  T acc[C][D];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) acc[c][q] = T(0);
#pragma unroll 1
  for (int j = 0; j < 27; ++j) {
    const int jx = j % 3, jy = (j / 3) % 3, jz = j / 9;
    const int id = L.node_map[wrapm(x + jx - 1, N) + N * (wrapm(y + jy - 1, N) + N * wrapm(z + jz - 1, N))];
    T cj[D][D];
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) cj[q][q2] = T(0);
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
      const int dx = jx - (k & 1), dy = jy - ((k >> 1) & 1), dz = jz - (k >> 2);
      if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) continue;  // j is not a corner of element k
      const T mk = (occ >> k) & 1u ? T(1) : T(0);
      const cptr<T> Kb = K + ((7 - k) * D) * M + (dx + 2 * dy + 4 * dz) * D;
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) cj[q][q2] = fma(mk, Kb[q * M + q2], cj[q][q2]);
    }
    if (id >= 0) {
      T v[C][D];
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) v[c][q2] = u[vix(c, n, id, D, q2)];
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2)
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c][q] = fma(cj[q][q2], v[c][q2], acc[c][q]);
    }
  }
  epilogue_node<T, EPI, C, D>(e, u, n, i, 0, &acc[0][0], nullptr, nullptr);
}

// Level 1, boundary nodes, as a masked stencil assembled in registers: the
// block of neighbour j is the sum of the K_e blocks of the active octant
// elements that contain both the node and j; every K_e entry is a symmetry-class
// value (wave-uniform, loaded once) with a compile-time sign, so the assembly
// is straight-line FMAs with the per-lane 0/1 occupancy factors and no memory
// traffic.  A thread takes C consecutive cases (grid row y: cases y*C ..),
// gathering each neighbour once for them.  The
// neighbour loads are issued from a clamped index and the values of an
// inactive neighbour (whose block is zero) are selected away, so no load sits
// in a branch.
// The grid is 1-D, rows workgroups per block of kBlock nodes, one per group
// of C cases, adjacent in the launch order: the rows of a node block run
// together and share its neighbour-id rows and occupancy in L2.
template <typename T, int D, int C, int EPI, int PRE = 0>
__global__ __launch_bounds__(kBlock) void k_apply_boundary_cls(LevelView<T> L, const T* __restrict__ u, EpiArgs<T> e,
                                                               int rows) {
  const int bi = block_index(L.xcd);
  const int t = (bi / rows) * kBlock + threadIdx.x;
  const int c0 = (bi % rows) * C;  // this workgroup's first case
  if (t >= L.n_bnd) return;
  const int i = L.boundary[t];
  const size_t n = (size_t)L.n_n;
  const unsigned occ = L.occ8[i];
  constexpr int NK = D == 1 ? 4 : 14;
  T kc[NK];
#pragma unroll
  for (int c = 0; c < NK; ++c) kc[c] = L.kcls[c];
  int nb[kBndStride];
  {
    const int4* row = reinterpret_cast<const int4*>(L.bnd_nbrs + (size_t)t * kBndStride);
#pragma unroll
    for (int k = 0; k < kBndStride / 4; ++k) {
      const int4 v = row[k];
      nb[4 * k] = v.x;
      nb[4 * k + 1] = v.y;
      nb[4 * k + 2] = v.z;
      nb[4 * k + 3] = v.w;
    }
  }
  T mk[8], mkn[8];
  if (L.oscale) {  // density hierarchy: the octant elements' stiffness scales (0 where inactive)
#pragma unroll
    for (int k = 0; k < 8; ++k) mk[k] = L.oscale[(size_t)i * 8 + k];
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) mk[k] = (occ >> k) & 1u ? T(1) : T(0);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) mkn[k] = -mk[k];
  T acc[C][D];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) acc[c][q] = T(0);
  // PRE: every neighbour's values are loaded before the assembly starts
  T w[PRE ? 27 : 1][C][D];
  if constexpr (PRE) {
#pragma unroll
    for (int j = 0; j < 27; ++j) {
      const size_t id = nb[j] >= 0 ? nb[j] : 0;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) w[j][c][q2] = u[vix(c0 + c, n, id, D, q2)];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the scheduler from sinking the loads into the assembly
  }
#pragma unroll
  for (int j = 0; j < 27; ++j) {
    const int jx = j % 3, jy = (j / 3) % 3, jz = j / 9;
    T cj[D][D];
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) cj[q][q2] = T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = jx - (k & 1), dy = jy - ((k >> 1) & 1), dz = jz - (k >> 2);
      if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) continue;  // j is not a corner of element k
      const int a = 7 - k, m = dx + 2 * dy + 4 * dz;
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2)
          cj[q][q2] = fma(kcls_negative<D>(a, q, q2) ? mkn[k] : mk[k], kc[kcls_index<D>(a ^ m, q, q2)], cj[q][q2]);
    }
    const bool act = nb[j] >= 0;
    const size_t id = act ? nb[j] : 0;
    T v[C][D];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) v[c][q2] = PRE ? w[PRE ? j : 0][c][q2] : u[vix(c0 + c, n, id, D, q2)];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) v[c][q2] = act ? v[c][q2] : T(0);
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c][q] = fma(cj[q][q2], v[c][q2], acc[c][q]);
  }
  epilogue_node<T, EPI, C, D>(e, u, n, i, c0, &acc[0][0], nullptr, nullptr);
}

// Level 1, boundary nodes, all C cases per thread: the masked stencil block
// of each neighbour is assembled once per node (not once per case) and the
// neighbour table row is read once.  The C x D values of neighbour j + 1 are
// loaded while neighbour j is assembled and applied (two register buffers);
// a scheduling barrier per neighbour keeps the compiler from hoisting the
// loads of all 27 neighbours (27 x C x D live values would spill).
template <typename T, int D, int C, int EPI>
__global__ __launch_bounds__(kBlock) void k_apply_boundary_all(LevelView<T> L, const T* __restrict__ u, EpiArgs<T> e) {
  const int t = block_index(L.xcd) * kBlock + threadIdx.x;
  if (t >= L.n_bnd) return;
  const int i = L.boundary[t];
  const size_t n = (size_t)L.n_n;
  const unsigned occ = L.occ8[i];
  constexpr int NK = D == 1 ? 4 : 14;
  const cptr<T> kcp = as_const(L.kcls);
  T kc[NK];
#pragma unroll
  for (int c = 0; c < NK; ++c) kc[c] = kcp[c];
  int nb[kBndStride];
  {
    const int4* row = reinterpret_cast<const int4*>(L.bnd_nbrs + (size_t)t * kBndStride);
#pragma unroll
    for (int k = 0; k < kBndStride / 4; ++k) {
      const int4 v = row[k];
      nb[4 * k] = v.x;
      nb[4 * k + 1] = v.y;
      nb[4 * k + 2] = v.z;
      nb[4 * k + 3] = v.w;
    }
  }
  T mk[8];
  if (L.oscale) {
#pragma unroll
    for (int k = 0; k < 8; ++k) mk[k] = L.oscale[(size_t)i * 8 + k];
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) mk[k] = (occ >> k) & 1u ? T(1) : T(0);
  }
  T acc[C][D];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) acc[c][q] = T(0);
  T vb[2][C][D];
  {
    const size_t id = nb[0] >= 0 ? nb[0] : 0;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) vb[0][c][q2] = u[vix(c, n, id, D, q2)];
  }
#pragma unroll
  for (int j = 0; j < 27; ++j) {
    const int cur = j & 1;
    if (j + 1 < 27) {
      const size_t id = nb[j + 1] >= 0 ? nb[j + 1] : 0;
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) vb[cur ^ 1][c][q2] = u[vix(c, n, id, D, q2)];
    }
    const int jx = j % 3, jy = (j / 3) % 3, jz = j / 9;
    T cj[D][D];
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) cj[q][q2] = T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = jx - (k & 1), dy = jy - ((k >> 1) & 1), dz = jz - (k >> 2);
      if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) continue;  // j is not a corner of element k
      const int a = 7 - k, m = dx + 2 * dy + 4 * dz;
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) {
          const T w = kc[kcls_index<D>(a ^ m, q, q2)];
          cj[q][q2] = fma(mk[k], kcls_negative<D>(a, q, q2) ? -w : w, cj[q][q2]);
        }
    }
    const T act = nb[j] >= 0 ? T(1) : T(0);
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
      for (int q2 = 0; q2 < D; ++q2) cj[q][q2] *= act;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) acc[c][q] = fma(cj[q][q2], vb[cur][c][q2], acc[c][q]);
    __builtin_amdgcn_sched_barrier(0);
  }
  epilogue_node<T, EPI, C, D>(e, u, n, i, 0, &acc[0][0], nullptr, nullptr);
}

// Level 1, boundary nodes: element-by-element over the active octant
// elements (occupancy bits), shared K_e with wave-uniform coefficients.  The 8
// corner values of an element are loaded inside that element's branch, which
// keeps the live register set to one element.
template <typename T, int D, int EPI>
__global__ __launch_bounds__(kBlock) void k_apply_boundary(LevelView<T> L, int C, const T* __restrict__ u, EpiArgs<T> e) {
  const int t = block_index(L.xcd) * kBlock + threadIdx.x;
  if (t >= L.n_bnd) return;
  const int i = L.boundary[t];
  const int N = L.N;
  const size_t n = (size_t)L.n_n;
  const int lin = L.node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  int nb[27];
  neighbour_ids<false>(L.node_map, N, x, y, z, nb);
  const unsigned occ = L.occ8[i];
  constexpr int M = 8 * D;
  T dv[D];
#pragma unroll
  for (int q = 0; q < D; ++q) dv[q] = needs_dinv<EPI>() ? e.dinv[(size_t)i * D + q] : T(0);
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    const cptr<T> K = as_const(L.K + (c & L.zero));  // (see k_apply_interior_run)
    T acc[D];
#pragma unroll
    for (int q = 0; q < D; ++q) acc[q] = T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (occ & (1u << k)) {
        const int a = 7 - k;
        const int ak = k & 1, bk = (k >> 1) & 1, ck = (k >> 2) & 1;
        T ue[8][D];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          // corners of an active element are active: nb >= 0
          const int j = (ak + (m & 1)) + 3 * (bk + ((m >> 1) & 1)) + 9 * (ck + ((m >> 2) & 1));
#pragma unroll
          for (int q = 0; q < D; ++q) ue[m][q] = u[vix(c, n, nb[j], D, q)];
        }
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
          for (int q = 0; q < D; ++q)
#pragma unroll
            for (int q2 = 0; q2 < D; ++q2) acc[q] = fma(K[(a * D + q) * M + m * D + q2], ue[m][q2], acc[q]);
      }
    }
    epilogue_node<T, EPI, 1, D>(e, u, n, i, c, acc, nullptr, dv);
  }
}

// Levels >= 2: per-element matrices (mask table or stored), element ids from
// the dense element map.  All index loads (27 neighbour ids, 8 element ids) are
// issued up front and the element/corner loops are unrolled, so the gathers of
// the 64 (element, corner) blocks are independent and overlap in flight; the
// D x D coefficient block of a corner is loaded once for the CB cases a thread
// owns (CB = c, or 1 with one grid row per case on small levels).
// NM (neighbour-major): the block of each of the 27 neighbours is first summed
// over the elements that contain both nodes, then the neighbour's values are
// gathered once for the CB cases — 27 gathers per case instead of one per
// (element, corner) pair (64), the sweep cost following the number of memory
// instructions.  An inactive element enters with weight 0 (its loads read a
// valid matrix), an inactive neighbour with a zero block.
template <typename T, int D, int CB, int KIND, int EPI, int BS, int NM = 0>
__global__ __launch_bounds__(BS) void k_apply_coarse(LevelView<T> L, const T* __restrict__ u, EpiArgs<T> e) {
  const int row = block_index(L.xcd) * BS + threadIdx.x;
  if (row >= (L.list ? L.n_list : L.n_n)) return;
  const int i = L.list ? L.list[row] : row;
  const int c0 = (int)blockIdx.y * CB;  // this thread's cases: c0 .. c0 + CB - 1
  const int N = L.N;
  const size_t n = (size_t)L.n_n;
  const int lin = L.node_lin[i];
  const int x = lin % N;
  const int t = lin / N;
  const int y = t % N;
  const int z = t / N;
  int nb[27];
  neighbour_ids<false>(L.node_map, N, x, y, z, nb);
  const int xm = wrapm(x - 1, N), ym = wrapm(y - 1, N), zm = wrapm(z - 1, N);
  int eid[8];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    eid[k] = L.elem_map[((k & 1) ? x : xm) + N * ((((k >> 1) & 1) ? y : ym) + N * ((k >> 2) ? z : zm))];
  T acc[CB][D];
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int q = 0; q < D; ++q) acc[c][q] = T(0);
  constexpr int M = 8 * D;
  if constexpr (NM) {
    const T* Kk[8];
    T mk[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool act = eid[k] >= 0;
      mk[k] = act ? T(1) : T(0);
      const int ek = act ? eid[k] : 0;
      if constexpr (KIND == KIND_TABLE)
        Kk[k] = L.K + (size_t)(act ? L.cmask[ek] : 0) * M * M + (7 - k) * D * M;
      else
        Kk[k] = L.K + (size_t)ek * M * M + (7 - k) * D * M;
    }
#pragma unroll
    for (int j = 0; j < 27; ++j) {
      const int jx = j % 3, jy = (j / 3) % 3, jz = j / 9;
      T cj[D][D];
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) cj[q][q2] = T(0);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int dx = jx - (k & 1), dy = jy - ((k >> 1) & 1), dz = jz - (k >> 2);
        if (dx < 0 || dx > 1 || dy < 0 || dy > 1 || dz < 0 || dz > 1) continue;  // j is not a corner of element k
        const int m = dx + 2 * dy + 4 * dz;
#pragma unroll
        for (int q = 0; q < D; ++q)
#pragma unroll
          for (int q2 = 0; q2 < D; ++q2) cj[q][q2] = fma(mk[k], Kk[k][q * M + m * D + q2], cj[q][q2]);
      }
      const size_t id = nb[j] >= 0 ? nb[j] : 0;
#pragma unroll
      for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) {
          const T v = u[vix(c0 + c, n, id, D, q2)];
#pragma unroll
          for (int q = 0; q < D; ++q) acc[c][q] = fma(cj[q][q2], v, acc[c][q]);
        }
    }
    epilogue_node<T, EPI, CB, D>(e, u, n, i, c0, &acc[0][0], nullptr, nullptr);
    return;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (eid[k] < 0) continue;
    const int ak = k & 1, bk = (k >> 1) & 1, ck = (k >> 2) & 1;
    const T* __restrict__ Km;
    if constexpr (KIND == KIND_TABLE)
      Km = L.K + (size_t)L.cmask[eid[k]] * M * M;
    else
      Km = L.K + (size_t)eid[k] * M * M;
    Km += (7 - k) * D * M;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      // corners of an active element are active: nb >= 0
      const int id = nb[(ak + (m & 1)) + 3 * (bk + ((m >> 1) & 1)) + 9 * (ck + ((m >> 2) & 1))];
      T coef[D][D];
#pragma unroll
      for (int q = 0; q < D; ++q)
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) coef[q][q2] = Km[q * M + m * D + q2];
#pragma unroll
      for (int c = 0; c < CB; ++c) {
#pragma unroll
        for (int q2 = 0; q2 < D; ++q2) {
          const T v = u[vix(c0 + c, n, id, D, q2)];
#pragma unroll
          for (int q = 0; q < D; ++q) acc[c][q] = fma(coef[q][q2], v, acc[c][q]);
        }
      }
    }
  }
  epilogue_node<T, EPI, CB, D>(e, u, n, i, c0, &acc[0][0], nullptr, nullptr);
}

// dst = src / sqrt(*nrm2), the squared norm read on the device; a zero or
// non-finite norm leaves a zero vector (the caller's estimate then fails).
template <typename T>
__global__ void k_normalize(size_t n, const T* __restrict__ src, const double* __restrict__ nrm2,
                            T* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double v = *nrm2;
  dst[i] = (v > 0.0 && v < INFINITY) ? T(double(src[i]) / sqrt(v)) : T(0);
}

// First smoothing step from a zero iterate: u = scale * D^-1 f (K 0 = 0).
template <typename T>
__global__ void k_smooth_zero(int n, int D, int C, const T* __restrict__ f, const T* __restrict__ dinv,
                              T scale, T* __restrict__ out, T* __restrict__ dvec) {
  // grid row = case (32-bit index arithmetic within a case)
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n * D) return;
  const size_t idx = (size_t)blockIdx.y * n * D + j;
  const T v = scale * dinv[j] * f[idx];
  out[idx] = v;
  if (dvec) dvec[idx] = v;
}

// ---------------------------------------------------------------- transfers (App. E.2)

// Restriction in gather form: coarse node X collects the fine nodes 2X + delta,
// delta in {-1,0,1}^3, with weight prod_d (1 - |delta_d|/2): exactly R = P^T.
// The 27 fine ids are looked up first; then, case by case, the 27 fine values
// are all loaded before the first FMA (27 gathers in flight instead of one
// dependent lookup-and-load per neighbour).  The sum runs over the neighbours
// in the same order either way; absent neighbours are skipped, not added as 0.
template <typename T, int Q, int D>
__global__ __launch_bounds__(kBlock) void k_restrict(LevelView<T> F, LevelView<T> Cv, const T* __restrict__ rf,
                                                     T* __restrict__ fc) {
  constexpr int C = Q / D;
  const int J = xcd_block() * kBlock + threadIdx.x;
  if (J >= Cv.n_n) return;
  const int Nc = Cv.N, Nf = F.N;
  const size_t nf = (size_t)F.n_n, nc = (size_t)Cv.n_n;
  const int lin = Cv.node_lin[J];
  const int X = lin % Nc;
  const int t = lin / Nc;
  const int Y = t % Nc;
  const int Z = t / Nc;
  int ids[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) {
    const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
    ids[k] = F.node_map[wrapm(2 * X + dx, Nf) + Nf * (wrapm(2 * Y + dy, Nf) + Nf * wrapm(2 * Z + dz, Nf))];
  }
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    T v[27][D];
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const size_t id = ids[k] >= 0 ? (size_t)ids[k] : 0;
#pragma unroll
      for (int d = 0; d < D; ++d) v[k][d] = rf[vix(c, nf, id, D, d)];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the FMA chain
    T acc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] = T(0);
#pragma unroll
    for (int k = 0; k < 27; ++k) {
      const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
      const T w = T((dx ? 0.5 : 1.0) * (dy ? 0.5 : 1.0) * (dz ? 0.5 : 1.0));
#pragma unroll
      for (int d = 0; d < D; ++d) acc[d] = ids[k] >= 0 ? fma(w, v[k][d], acc[d]) : acc[d];
    }
#pragma unroll
    for (int d = 0; d < D; ++d) fc[vix(c, nc, J, D, d)] = acc[d];
  }
}

// Prolongation + correction: u_f(i) += sum_k W_ik u_c(I_ik) (App. E.1 weights).
// Per axis an even fine coordinate has one parent (weight 1), an odd one two
// (1/2 each).  The up to 8 parent ids are looked up first; then, case by case,
// the parents' values are loaded before the first FMA.  The sum runs over the
// parents in the same order as a loop over (z, y, x) offsets would.
template <typename T, int Q, int D>
__global__ __launch_bounds__(kBlock) void k_prolong_add(LevelView<T> F, LevelView<T> Cv, const T* __restrict__ uc,
                                                        T* __restrict__ uf) {
  constexpr int C = Q / D;
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= F.n_n) return;
  const int Nc = Cv.N, Nf = F.N;
  const size_t nf = (size_t)F.n_n, nc = (size_t)Cv.n_n;
  const int lin = F.node_lin[i];
  const int x = lin % Nf;
  const int t = lin / Nf;
  const int y = t % Nf;
  const int z = t / Nf;
  const int cx0 = x >> 1, cy0 = y >> 1, cz0 = z >> 1;
  const int nx = (x & 1) ? 2 : 1, ny = (y & 1) ? 2 : 1, nz = (z & 1) ? 2 : 1;
  const T w = T(1.0 / (nx * ny * nz));
  int pid[8];  // parent (ox, oy, oz) = (k & 1, (k >> 1) & 1, k >> 2); -1 where absent
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ox = k & 1, oy = (k >> 1) & 1, oz = k >> 2;
    pid[k] = -1;
    if (ox < nx && oy < ny && oz < nz)  // (a consistent hierarchy has every such parent)
      pid[k] = Cv.node_map[wrapm(cx0 + ox, Nc) + Nc * (wrapm(cy0 + oy, Nc) + Nc * wrapm(cz0 + oz, Nc))];
  }
#pragma unroll 1
  for (int c = 0; c < C; ++c) {
    T acc[D], v[8][D];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] = uf[vix(c, nf, i, D, d)];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (pid[k] >= 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) v[k][d] = uc[vix(c, nc, pid[k], D, d)];
      }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (pid[k] >= 0) {
#pragma unroll
        for (int d = 0; d < D; ++d) acc[d] = fma(w, v[k][d], acc[d]);
      }
#pragma unroll
    for (int d = 0; d < D; ++d) uf[vix(c, nf, i, D, d)] = acc[d];
  }
}

// ---------------------------------------------------------------- coarsest solve

// u = Kinv f with Kinv the pinned inverse (symmetric, pinned rows/cols zero).
// A workgroup owns 64 DOF rows (node*D + d); its 4 waves split the columns
// (wave w takes columns w, w + 4, ..), so that four times as many column loads
// are in flight for the small coarsest systems, and add their FP64 partial
// sums through LDS at the end.  f (all C cases) is staged in LDS in chunks of
// kCoarseChunk DOFs, read by broadcast; the Kinv column reads (= rows by
// symmetry) are coalesced over the 64 rows.
constexpr int kCoarseChunk = 256;
constexpr int kCoarseSplit = 4;
template <typename T, int C>
__global__ __launch_bounds__(64 * kCoarseSplit) void k_coarse_solve(const T* __restrict__ Kinv, int cn, int D,
                                                                   const T* __restrict__ f, T* __restrict__ u) {
  __shared__ T fs[kCoarseChunk * C];
  __shared__ double part[kCoarseSplit - 1][C][64];
  const int n = cn / D;
  const int lane = threadIdx.x & 63, split = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + lane;
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  for (int j0 = 0; j0 < cn; j0 += kCoarseChunk) {
    const int m = min(kCoarseChunk, cn - j0);
    __syncthreads();
    for (int k = threadIdx.x; k < m * C; k += 64 * kCoarseSplit) {
      const int j = j0 + k / C, c = k % C;
      fs[k] = f[vix(c, n, j / D, D, j % D)];
    }
    __syncthreads();
    if (row < cn) {
#pragma unroll 4
      for (int jj = split; jj < m; jj += kCoarseSplit) {
        const double kv = (double)Kinv[(size_t)(j0 + jj) * cn + row];
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += kv * (double)fs[jj * C + c];
      }
    }
  }
  if (split > 0) {
#pragma unroll
    for (int c = 0; c < C; ++c) part[split - 1][c][lane] = acc[c];
  }
  __syncthreads();
  if (split > 0 || row >= cn) return;
#pragma unroll
  for (int s2 = 0; s2 < kCoarseSplit - 1; ++s2)
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] += part[s2][c][lane];
  const int node = row / D, q = row % D;
#pragma unroll
  for (int c = 0; c < C; ++c) u[vix(c, n, node, D, q)] = (T)acc[c];
}

// Layout changes between the ABI's [n][Q] and the solver's [Q][n].
// ABI [n][C][D] -> solver [C][n][D]
template <typename Tin, typename Tout>
__global__ void k_aos_to_soa(const Tin* __restrict__ a, Tout* __restrict__ b, int n, int C, int D) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;  // index into b
  if (idx >= (size_t)n * C * D) return;
  const int d = (int)(idx % D);
  const size_t t = idx / D;
  const size_t i = t % n, c = t / n;
  b[idx] = (Tout)a[(i * C + c) * D + d];
}

// solver [C][n][D] -> ABI [n][C][D]
template <typename Tin, typename Tout>
__global__ void k_soa_to_aos(const Tin* __restrict__ a, Tout* __restrict__ b, int n, int C, int D) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;  // index into b
  if (idx >= (size_t)n * C * D) return;
  const int d = (int)(idx % D);
  const size_t t = idx / D;
  const size_t c = t % C, i = t / C;
  b[idx] = (Tout)a[(c * n + i) * D + d];
}

// ---------------------------------------------------------------- vector kernels

template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ a, Tout* __restrict__ b, size_t n) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = (Tout)a[i];
}

template <typename T>
__global__ void k_inv(const T* __restrict__ a, T* __restrict__ b, size_t n) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = a[i] != T(0) ? T(1) / a[i] : T(0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block reduction of NV values per thread -> partial[block][NV]; fixed order.
template <int NV>
__device__ void block_reduce_store(double (&v)[NV], double* __restrict__ partial) {
  __shared__ double sh[kBlock / 64][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) sh[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += sh[w][threadIdx.x];
    partial[(size_t)blockIdx.x * NV + threadIdx.x] = s;
  }
}

// CB: b enters with its column means removed, b - (T)(sums[col] inv_n), rounded
// as k_sub_mean rounds it (the dot of a projected vector without writing it)
template <typename T, int C, int D, bool CB = false>
__global__ __launch_bounds__(kBlock) void k_dot(const T* __restrict__ a, const T* __restrict__ b, int n,
                                                double* __restrict__ partial, const double* __restrict__ sums = nullptr,
                                                double inv_n = 0.0) {
  double v[C];
#pragma unroll
  for (int c = 0; c < C; ++c) v[c] = 0.0;
  T m[CB ? C * D : 1];
  if constexpr (CB) {
#pragma unroll
    for (int k = 0; k < C * D; ++k) m[k] = (T)(sums[k] * inv_n);
  }
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const size_t idx = vix(c, n, i, D, q);
        T bv = b[idx];
        if constexpr (CB) bv -= m[c * D + q];
        v[c] += (double)a[idx] * (double)bv;
      }
  }
  block_reduce_store<C>(v, partial);
}

// p.q per case and the column sums of q, in one pass over p and q
template <typename T, int C, int D>
__global__ __launch_bounds__(kBlock) void k_dot_colsum(const T* __restrict__ a, const T* __restrict__ b, int n,
                                                       double* __restrict__ partial) {
  double v[C + C * D];
#pragma unroll
  for (int k = 0; k < C + C * D; ++k) v[k] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const size_t idx = vix(c, n, i, D, q);
        const double bv = (double)b[idx];
        v[c] += (double)a[idx] * bv;
        v[C + c * D + q] += bv;
      }
  }
  block_reduce_store<C + C * D>(v, partial);
}

// r.(z - its column means) and r.r per case, in one pass over r and z
template <typename T, int C, int D>
__global__ __launch_bounds__(kBlock) void k_dot2_centered(const T* __restrict__ r, const T* __restrict__ z, int n,
                                                          const double* __restrict__ sums, double inv_n,
                                                          double* __restrict__ partial) {
  double v[2 * C];
#pragma unroll
  for (int k = 0; k < 2 * C; ++k) v[k] = 0.0;
  T m[C * D];
#pragma unroll
  for (int k = 0; k < C * D; ++k) m[k] = (T)(sums[k] * inv_n);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < D; ++q) {
        const size_t idx = vix(c, n, i, D, q);
        const double rv = (double)r[idx];
        const T zv = z[idx] - m[c * D + q];
        v[c] += rv * (double)zv;
        v[C + c] += rv * rv;
      }
  }
  block_reduce_store<2 * C>(v, partial);
}

template <typename Ta, typename Tb, int C, int D>
__global__ __launch_bounds__(kBlock) void k_gram(const Ta* __restrict__ a, const Tb* __restrict__ b, int n,
                                                 double* __restrict__ partial) {
  double v[C * C];
#pragma unroll
  for (int c = 0; c < C * C; ++c) v[c] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double av[C][D], bv[C][D];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
      for (int q = 0; q < D; ++q) {
        av[c][q] = (double)a[vix(c, n, i, D, q)];
        bv[c][q] = (double)b[vix(c, n, i, D, q)];
      }
#pragma unroll
    for (int c1 = 0; c1 < C; ++c1)
#pragma unroll
      for (int c2 = 0; c2 < C; ++c2)
#pragma unroll
        for (int q = 0; q < D; ++q) v[c1 * C + c2] += av[c1][q] * bv[c2][q];
  }
  block_reduce_store<C * C>(v, partial);
}

// Column sums over nodes: partial[block][q] = sum_i v[q][i] (FP64 accumulation).
template <typename T, int Q, int D>
__global__ __launch_bounds__(kBlock) void k_colsum(const T* __restrict__ v, int n, double* __restrict__ partial) {
  double acc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] += (double)v[vix(q / D, n, i, D, q % D)];
  }
  block_reduce_store<Q>(acc, partial);
}

// v[q][i] -= sums[q] / n : removes the rigid-translation (constant) component.
// Grid row = case, 32-bit index arithmetic within a case.
template <typename T>
__global__ void k_sub_mean(T* __restrict__ v, int n, int D, const double* __restrict__ sums, double inv_n) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n * D) return;
  const int c = blockIdx.y;
  v[(size_t)c * n * D + j] -= (T)(sums[c * D + j % D] * inv_n);
}

template <typename T>
__global__ void k_axpby(T* __restrict__ y, const T* __restrict__ x, T alpha, T beta, size_t n) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = alpha * x[i] + beta * y[i];
}

template <typename T>
__global__ void k_scale_add_comp(T* __restrict__ y, const T* __restrict__ x, T alpha, const double* __restrict__ add,
                                 int n, int D, size_t total) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const size_t c = i / ((size_t)n * D);
  y[i] = alpha * x[i] + (T)add[c * D + i % D];
}

template <typename T>
__global__ void k_mul_nodewise(T* __restrict__ v, const T* __restrict__ w, int n, int D, int divide, size_t total) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  const size_t node = (i / D) % n;
  const T ww = w[node * D + i % D];
  v[i] = divide ? v[i] / ww : v[i] * ww;
}

// Second stage with the values split over two outputs: k < n1 -> out1[k], else out2[k - n1].
__global__ void k_reduce_split(const double* __restrict__ partial, int nblocks, int nv, int n1, double* __restrict__ out1,
                               double* __restrict__ out2) {
  __shared__ double sh[kBlock];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partial[(size_t)b * nv + k];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (k < n1)
      out1[k] = sh[0];
    else
      out2[k - n1] = sh[0];
  }
}

// Second stage: out[k] = sum over blocks of partial[b][k], fixed order.
// One workgroup per reduced value k (grid = nv).
__global__ void k_reduce_final(const double* __restrict__ partial, int nblocks, int nv, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  {
    const int k = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partial[(size_t)b * nv + k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
  }
}

// u += alpha p, r -= alpha q; with qsums, q enters with its column means removed,
// so a residual with zero column means keeps them zero
// the D column means of case row c of a [C][n][D] vector, rounded to T (zero without sums)
template <typename T, int D>
__device__ __forceinline__ void case_means(const double* __restrict__ sums, double inv_n, int c, T (&m)[D]) {
#pragma unroll
  for (int d = 0; d < D; ++d) m[d] = sums ? (T)(sums[c * D + d] * inv_n) : T(0);
}

template <typename T, int D>
__global__ void k_pcg_update(T* __restrict__ u, T* __restrict__ r, const T* __restrict__ p,
                             const T* __restrict__ q, const double* __restrict__ alpha, int n,
                             const double* __restrict__ qsums, double inv_n) {
  // grid row = case
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n * D) return;
  const size_t i = (size_t)blockIdx.y * n * D + j;
  const T a = (T)alpha[blockIdx.y];
  T m[D];
  case_means<T, D>(qsums, inv_n, blockIdx.y, m);
  u[i] = fma(a, p[i], u[i]);
  r[i] = fma(-a, q[i] - m[j % D], r[i]);
}

// p = z + beta p; with sums, z enters with its column means removed (as k_sub_mean
// would have written it)
template <typename T, int D>
__global__ void k_pcg_direction(T* __restrict__ p, const T* __restrict__ z, const double* __restrict__ beta, int n,
                                const double* __restrict__ sums, double inv_n) {
  // grid row = case
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n * D) return;
  const size_t i = (size_t)blockIdx.y * n * D + j;
  const T b = (T)beta[blockIdx.y];
  T m[D];
  case_means<T, D>(sums, inv_n, blockIdx.y, m);
  p[i] = fma(b, p[i], z[i] - m[j % D]);
}

// stop (nullable): the device-side convergence flag of captured PCG blocks; once
// set, alpha = beta = 0 and the remaining iterations of a block change nothing
__global__ void k_pcg_alpha(const double* rz, const double* pq, double* alpha, int C, const double* stop) {
  int c = threadIdx.x;
  const bool off = stop && *stop != 0.0;
  if (c < C) alpha[c] = (!off && pq[c] > 0.0 && isfinite(rz[c] / pq[c])) ? rz[c] / pq[c] : 0.0;
}

__global__ void k_pcg_beta(const double* rz_new, double* rz, double* beta, int C, const double* stop) {
  int c = threadIdx.x;
  if (c < C) {
    if (stop && *stop != 0.0) {
      beta[c] = 0.0;
      return;
    }
    beta[c] = (rz[c] != 0.0 && isfinite(rz_new[c] / rz[c])) ? rz_new[c] / rz[c] : 0.0;
    rz[c] = rz_new[c];
  }
}

// End of a captured PCG iteration: flags[1] counts the iterations that ran with
// the flag clear; flags[0] is set once every case meets ||r_m||^2 <= flags[2 + m]
// (the squared target) or a residual is not finite (the host reports that).
__global__ void k_pcg_check(const double* rr, int C, double* flags) {
  if (threadIdx.x != 0 || flags[0] != 0.0) return;
  flags[1] += 1.0;
  bool done = true;
  for (int c = 0; c < C; ++c) {
    if (!isfinite(rr[c])) {
      done = true;
      break;
    }
    if (!(rr[c] <= flags[2 + c])) done = false;
  }
  if (done) flags[0] = 1.0;
}

template <typename T>
__global__ void k_copy_node(const T* __restrict__ u, int n, int Q, int D, T* __restrict__ tmp) {
  const int q = threadIdx.x;
  if (q < Q) tmp[q] = u[vix(q / D, n, 0, D, q % D)];
}

template <typename T>
__global__ void k_sub_node(T* __restrict__ u, size_t total, int n, int D, const T* __restrict__ tmp) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < total) u[i] -= tmp[(i / ((size_t)n * D)) * D + i % D];
}

template <typename T>
__global__ void k_accumulate(double* __restrict__ u, const T* __restrict__ d, size_t n, double a) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) u[i] += a * (double)d[i];
}

// ---------------------------------------------------------------- hierarchy construction

__global__ void k_voxel_flags(const uint8_t* __restrict__ vox, size_t n, int* __restrict__ flags) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) flags[i] = vox[i] != 0;
}

// node (x,y,z) active iff element (x-a, y-b, z-c) is active for some corner (a,b,c)
// (vertex union of eq. gmgcoarsenode); input: dense element map (>= 0 active)
__global__ void k_node_flags(const int* __restrict__ emap, int N, int* __restrict__ nflags) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)N * N * N;
  if (i >= n) return;
  const int x = (int)(i % N), y = (int)((i / N) % N), z = (int)(i / ((size_t)N * N));
  int f = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ex = wrapm(x - (k & 1), N), ey = wrapm(y - ((k >> 1) & 1), N), ez = wrapm(z - ((k >> 2) & 1), N);
    f |= emap[ex + N * (ey + N * ez)] >= 0;
  }
  nflags[i] = f;
}

// coarse voxel (I,J,K) active iff any child (2I+a, 2J+b, 2K+c) is active; the
// child pattern is kept as a mask byte (bit a+2b+4c)
__global__ void k_coarsen(const int* __restrict__ femap, int Nf, int* __restrict__ cflags,
                          uint8_t* __restrict__ dcmask) {
  const int Nc = Nf / 2;
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t n = (size_t)Nc * Nc * Nc;
  if (i >= n) return;
  const int X = (int)(i % Nc), Y = (int)((i / Nc) % Nc), Z = (int)(i / ((size_t)Nc * Nc));
  unsigned m = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int fx = 2 * X + (c & 1), fy = 2 * Y + ((c >> 1) & 1), fz = 2 * Z + ((c >> 2) & 1);
    if (femap[fx + Nf * (fy + Nf * fz)] >= 0) m |= 1u << c;
  }
  cflags[i] = m != 0;
  dcmask[i] = (uint8_t)m;
}

// --- scan: 256 threads x 16 items per block
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

// The same for NT threads, with the NT / 64 wave sums in the caller's LDS
// (free at the call; it is free again when the function returns).
template <int NT>
__device__ int block_exclusive_scan_n(int v, int* total, int* wsum) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int tt = __shfl_up(incl, o, 64);
    if (lane >= o) incl += tt;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

__device__ int block_exclusive_scan(int v, int* total) {
  __shared__ int wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int tt = __shfl_up(incl, o, 64);
    if (lane >= o) incl += tt;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wid) off += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

__global__ void k_scan_reduce(const int* __restrict__ flags, size_t n, int* __restrict__ bsum) {
  const size_t base = (size_t)blockIdx.x * kScanTile;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    size_t i = base + (size_t)k * kBlock + threadIdx.x;
    if (i < n) s += flags[i];
  }
  int tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of nb block sums by one block; total -> *d_total
__global__ void k_scan_top(int* __restrict__ bsum, int nb, int* __restrict__ d_total) {
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += kBlock) {
    const int i = base + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int tot;
    const int ex = block_exclusive_scan(v, &tot);
    const int c0 = carry;
    if (i < nb) bsum[i] = c0 + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = c0 + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *d_total = carry;
}

// Tables of the staged interior sweep, one workgroup per 256 interior nodes:
// the 27 x 256 neighbour ids are sorted in LDS (bitonic), the distinct ones
// counted (pass 0, every workgroup b: cnt[b]) or, for the workgroups
// b = blk[g] the staged sweep takes, written out ascending at off[g] together
// with each node's 27 positions among them (pass 1: binary search).
template <int NB>
__global__ __launch_bounds__(NB) void k_stage_tables(const int* __restrict__ interior, int n_int,
                                                         const int* __restrict__ node_lin,
                                                         const int* __restrict__ node_map, int N, int pass,
                                                         const int* __restrict__ blk, int* __restrict__ cnt,
                                                         const long long* __restrict__ off, int* __restrict__ ids,
                                                         uint16_t* __restrict__ slot) {
  constexpr int kStageNodes = NB;
  constexpr int kStageSort = NB == 256 ? 8192 : 16384;  // >= 27 * NB, a power of two
  constexpr int kStageItems = kStageSort / NB;
  static_assert(27 * NB <= kStageSort, "sort buffer too small");
  __shared__ int s[kStageSort];
  const int g = blockIdx.x;
  const int b = pass == 0 ? g : blk[g];
  const int t = b * kStageNodes + (int)threadIdx.x;
  const bool valid = t < n_int;
  int nb[27];
  if (valid) {
    const int lin = node_lin[interior[t]];
    neighbour_ids<true>(node_map, N, lin % N, (lin / N) % N, lin / (N * N), nb);
  }
#pragma unroll
  for (int j = 0; j < 27; ++j) s[(int)threadIdx.x * 27 + j] = valid ? nb[j] : INT_MAX;
  for (int k = 27 * kStageNodes + (int)threadIdx.x; k < kStageSort; k += kStageNodes) s[k] = INT_MAX;
  __syncthreads();
  for (int size = 2; size <= kStageSort; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int p = (int)threadIdx.x; p < kStageSort / 2; p += kStageNodes) {
        const int lo = 2 * p - (p & (stride - 1));  // the partner index lo + stride has that bit set
        const int hi = lo + stride;
        const int a = s[lo], c = s[hi];
        if ((a > c) == ((lo & size) == 0)) {
          s[lo] = c;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  // distinct values: thread k owns the sorted entries k * kStageItems ..
  int v[kStageItems];
  int m = 0;
  const int base = (int)threadIdx.x * kStageItems;
#pragma unroll
  for (int k = 0; k < kStageItems; ++k) {
    v[k] = s[base + k];
    const int prev = base + k > 0 ? s[base + k - 1] : INT_MIN;
    if (v[k] == INT_MAX || v[k] == prev) v[k] = -1;  // not the first of its value
    m += v[k] >= 0;
  }
  int total;
  __syncthreads();  // every read of s above is done: its first words hold the wave sums
  int pos = block_exclusive_scan_n<kStageNodes>(m, &total, s);
  if (pass == 0) {
    if (threadIdx.x == 0) cnt[b] = total;
    return;
  }
  const long long o0 = off[b];
#pragma unroll
  for (int k = 0; k < kStageItems; ++k)
    if (v[k] >= 0) {
      s[pos] = v[k];
      ids[o0 + pos] = v[k];
      ++pos;
    }
  __syncthreads();
  if (!valid) return;
  uint16_t* row = slot + (size_t)t * kSlotStride;
#pragma unroll
  for (int j = 0; j < 27; ++j) {
    int lo = 0, hi = total;  // first position with s[pos] >= nb[j]
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s[mid] < nb[j]) lo = mid + 1;
      else hi = mid;
    }
    row[j] = (uint16_t)lo;
  }
  row[27] = 0;
}

// per block: ids of the flagged items in linear order; map (id or -1), lin (id -> index)
__global__ void k_scan_compact(const int* __restrict__ flags, size_t n, const int* __restrict__ boff,
                               int* __restrict__ map, int* __restrict__ lin) {
  const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    size_t i = base + k;
    v[k] = i < n ? flags[i] : 0;
    s += v[k];
  }
  int tot;
  int off = block_exclusive_scan(s, &tot) + boff[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    size_t i = base + k;
    if (i < n) {
      if (v[k]) {
        map[i] = off;
        if (lin) lin[off] = (int)i;
        ++off;
      } else {
        map[i] = -1;
      }
    }
  }
}

__global__ void k_occ8(const int* __restrict__ node_lin, int n_n, const int* __restrict__ emap, int N,
                       uint8_t* __restrict__ occ8) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_n) return;
  const int lin = node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  unsigned m = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ex = wrapm(x - 1 + (k & 1), N), ey = wrapm(y - 1 + ((k >> 1) & 1), N),
              ez = wrapm(z - 1 + ((k >> 2) & 1), N);
    if (emap[ex + N * (ey + N * ez)] >= 0) m |= 1u << k;
  }
  occ8[i] = (uint8_t)m;
}

// flags[i] = (occ8[i] == 255) == want_full
__global__ void k_occ_flags(const uint8_t* __restrict__ occ8, int n, int want_full, int* __restrict__ flags) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) flags[i] = ((occ8[i] == 255) ? 1 : 0) == want_full;
}

__global__ void k_gather_cmask(const int* __restrict__ elem_lin, int n_e, const uint8_t* __restrict__ dense,
                               uint8_t* __restrict__ cmask) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e < n_e) cmask[e] = dense[elem_lin[e]];
}

__global__ void k_elem_nodes(const int* __restrict__ elem_lin, int n_e, const int* __restrict__ node_map, int N,
                             int* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= n_e) return;
  const int lin = elem_lin[e];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int nx = wrapm(x + (k & 1), N), ny = wrapm(y + ((k >> 1) & 1), N), nz = wrapm(z + ((k >> 2) & 1), N);
    out[(size_t)e * 8 + k] = node_map[nx + N * (ny + N * nz)];
  }
}

// App. E.1: x_c = floor(x_f/2), corners (x_c + o_k) mod N_c, w_k = prod (1 - |xi - o|)
__global__ void k_prol_maps(const int* __restrict__ node_lin, int n_n, int Nf, const int* __restrict__ cmap,
                            int Nc, int* __restrict__ idx, double* __restrict__ w) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_n) return;
  const int lin = node_lin[i];
  const int x = lin % Nf, y = (lin / Nf) % Nf, z = lin / (Nf * Nf);
  const double xi[3] = {(x & 1) * 0.5, (y & 1) * 0.5, (z & 1) * 0.5};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int o[3] = {k & 1, (k >> 1) & 1, (k >> 2) & 1};
    double wk = 1.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) wk *= 1.0 - fabs(xi[d] - (double)o[d]);
    int id = -1;
    if (wk != 0.0) {
      const int X = wrapm((x >> 1) + o[0], Nc), Y = wrapm((y >> 1) + o[1], Nc), Z = wrapm((z >> 1) + o[2], Nc);
      id = cmap[X + Nc * (Y + Nc * Z)];
    }
    if (idx) idx[(size_t)i * 8 + k] = id;
    if (w) w[(size_t)i * 8 + k] = wk;
  }
}

// Local Galerkin projection (Sec. 4.6): K_E = sum_{active children c} P_c^T K_c P_c,
// P_c = Ps_c (8x8 trilinear weights) (x) I_D.  One block per coarse element.
template <int D>
__global__ __launch_bounds__(kBlock) void k_galerkin(const int* __restrict__ elem_lin_c, int Nc,
                                                     const int* __restrict__ emap_f,
                                                     const uint8_t* __restrict__ cmask_f,
                                                     const double* __restrict__ Ksrc, int src_kind,
                                                     const double* __restrict__ Ps,
                                                     const double* __restrict__ fscale, double* __restrict__ out64,
                                                     float* __restrict__ out32) {
  constexpr int M = 8 * D;
  __shared__ double Kc[M * M];
  __shared__ double T1[M * M];
  __shared__ double acc[M * M];
  __shared__ double P[64];
  const int e = blockIdx.x;
  const int Nf = 2 * Nc;
  const int lin = elem_lin_c[e];
  const int X = lin % Nc, Y = (lin / Nc) % Nc, Z = lin / (Nc * Nc);
  for (int t = threadIdx.x; t < M * M; t += kBlock) acc[t] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const int fx = 2 * X + (c & 1), fy = 2 * Y + ((c >> 1) & 1), fz = 2 * Z + ((c >> 2) & 1);
    const int fid = emap_f[fx + Nf * (fy + Nf * fz)];
    if (fid < 0) continue;  // uniform across the block
    const double* src = src_kind == KIND_SHARED ? Ksrc
                        : src_kind == KIND_TABLE ? Ksrc + (size_t)cmask_f[fid] * M * M
                                                 : Ksrc + (size_t)fid * M * M;
    const double sc = fscale ? fscale[fid] : 1.0;  // density hierarchy: the child's stiffness scale
    __syncthreads();
    for (int t = threadIdx.x; t < M * M; t += kBlock) Kc[t] = sc * src[t];
    if (threadIdx.x < 64) P[threadIdx.x] = Ps[c * 64 + threadIdx.x];
    __syncthreads();
    // T1[(m,i),(p,j)] = sum_n Kc[(m,i),(n,j)] P[n][p]
    for (int t = threadIdx.x; t < M * M; t += kBlock) {
      const int row = t / M, col = t % M;
      const int p = col / D, j = col % D;
      double s = 0.0;
#pragma unroll
      for (int n = 0; n < 8; ++n) s += Kc[row * M + n * D + j] * P[n * 8 + p];
      T1[t] = s;
    }
    __syncthreads();
    // acc[(o,i),(p,j)] += sum_m P[m][o] T1[(m,i),(p,j)]
    for (int t = threadIdx.x; t < M * M; t += kBlock) {
      const int row = t / M, col = t % M;
      const int o = row / D, i = row % D;
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < 8; ++m) s += P[m * 8 + o] * T1[(m * D + i) * M + col];
      acc[t] += s;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < M * M; t += kBlock) {
    out64[(size_t)e * M * M + t] = acc[t];
    out32[(size_t)e * M * M + t] = (float)acc[t];
  }
}

template <typename T, int D, int KIND>
__global__ void k_diagonal(LevelView<T> L, T* __restrict__ diag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= L.n_n) return;
  constexpr int M = 8 * D;
  const int N = L.N;
  const int lin = L.node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  T acc[D];
#pragma unroll
  for (int q = 0; q < D; ++q) acc[q] = T(0);
  for (int k = 0; k < 8; ++k) {
    const T* Km;
    T sc = T(1);
    if constexpr (KIND == KIND_SHARED) {
      if (!(L.occ8[i] & (1u << k))) continue;
      Km = L.K;
      if (L.oscale) sc = L.oscale[(size_t)i * 8 + k];
    } else {
      const int ex = wrapm(x - 1 + (k & 1), N), ey = wrapm(y - 1 + ((k >> 1) & 1), N),
                ez = wrapm(z - 1 + ((k >> 2) & 1), N);
      const int eid = L.elem_map[ex + N * (ey + N * ez)];
      if (eid < 0) continue;
      Km = KIND == KIND_TABLE ? L.K + (size_t)L.cmask[eid] * M * M : L.K + (size_t)eid * M * M;
    }
    const int a = 7 - k;
#pragma unroll
    for (int q = 0; q < D; ++q) acc[q] += sc * Km[(a * D + q) * M + a * D + q];
  }
#pragma unroll
  for (int q = 0; q < D; ++q) diag[(size_t)i * D + q] = acc[q];
}

// Every element matrix of a level as an explicit [n_e][M][M] array (export / coarsest assembly).
template <int D, int KIND>
__global__ void k_expand_elem(LevelView<double> L, int n_e, const int* __restrict__ elem_lin,
                              double* __restrict__ out) {
  constexpr int M = 8 * D;
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (size_t)n_e * M * M) return;
  const int e = (int)(t / (M * M));
  const int r = (int)(t % (M * M));
  double v;
  if constexpr (KIND == KIND_SHARED)
    v = L.K[r];
  else if constexpr (KIND == KIND_TABLE)
    v = L.K[(size_t)L.cmask[e] * M * M + r];
  else
    v = L.K[(size_t)e * M * M + r];
  out[t] = v;
}

// f_i = sum over active octant elements of the rows of f_e = K_e X0 at i's corner
// (density hierarchy: each octant element's rows weighted by its stiffness scale)
__global__ void k_load_vector(const int* __restrict__ node_lin, const uint8_t* __restrict__ occ8,
                              const double* __restrict__ oscale, int n_n, int D, int C, const double* __restrict__ fe,
                              double* __restrict__ f) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_n) return;
  const unsigned occ = occ8[i];
  for (int c = 0; c < C; ++c)
    for (int q = 0; q < D; ++q) {
      double s = 0.0;
      for (int k = 0; k < 8; ++k)
        if (occ & (1u << k)) s += (oscale ? oscale[(size_t)i * 8 + k] : 1.0) * fe[((7 - k) * D + q) * C + c];
      f[vix(c, n_n, i, D, q)] = s;
    }
}

// ---------------------------------------------------------------- density (SIMP) cells, App. F.3

__global__ void k_density_flags(const double* __restrict__ rho, size_t n, double prune, uint8_t* __restrict__ vox) {
  const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) vox[i] = rho[i] > prune ? 1 : 0;
}

__global__ void k_element_scale(const int* __restrict__ elem_lin, int n_e, const double* __restrict__ rho, double p,
                                double rho_min, double* __restrict__ erho, double* __restrict__ escale) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= n_e) return;
  const double r = rho[elem_lin[e]];
  erho[e] = r;
  escale[e] = rho_min + pow(r, p);
}

// o[i][k] = scale of octant element k of node i (element (x-1+a, y-1+b, z-1+c), k = a+2b+4c), 0 if inactive
__global__ void k_node_oscale(const int* __restrict__ node_lin, int n_n, const int* __restrict__ emap, int N,
                              const double* __restrict__ escale, double* __restrict__ o64, float* __restrict__ o32) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_n) return;
  const int lin = node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  for (int k = 0; k < 8; ++k) {
    const int ex = wrapm(x - 1 + (k & 1), N), ey = wrapm(y - 1 + ((k >> 1) & 1), N),
              ez = wrapm(z - 1 + ((k >> 2) & 1), N);
    const int eid = emap[ex + N * (ey + N * ez)];
    const double v = eid >= 0 ? escale[eid] : 0.0;
    o64[(size_t)i * 8 + k] = v;
    o32[(size_t)i * 8 + k] = (float)v;
  }
}

__global__ void k_iota(int* __restrict__ a, int n) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] = i;
}

// One thread per active element: d_j = X0_j - u_e,j (corner values of case j),
// y_j = K0 d_j, E_ij = d_i . y_j; dC[lin][i][j] = g E_ij and dJ[lin] = g sum_ij G_ij E_ij
// with g = p rho^(p-1) / N^3 (App. F.3).  u in the ABI layout [n][C][D].
template <int D, int C>
__global__ __launch_bounds__(kBlock) void k_simp_sensitivity(const int* __restrict__ elem_lin, int n_e,
                                                             const int* __restrict__ node_map, int N,
                                                             const double* __restrict__ u,
                                                             const double* __restrict__ Ke,
                                                             const double* __restrict__ X0,
                                                             const double* __restrict__ erho, double p,
                                                             const double* __restrict__ G, double* __restrict__ dJ,
                                                             double* __restrict__ dC) {
  constexpr int M = 8 * D;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= n_e) return;
  const int lin = elem_lin[e];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  int nd[8];
#pragma unroll
  for (int a = 0; a < 8; ++a)
    nd[a] = node_map[wrapm(x + (a & 1), N) + N * (wrapm(y + ((a >> 1) & 1), N) + N * wrapm(z + (a >> 2), N))];
  const cptr<double> K = as_const(Ke);
  const cptr<double> X = as_const(X0);
  double E[C][C];
#pragma unroll 1
  for (int j = 0; j < C; ++j) {
    double dj[M], yj[M];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int q = 0; q < D; ++q) dj[a * D + q] = X[(a * D + q) * C + j] - u[((size_t)nd[a] * C + j) * D + q];
#pragma unroll
    for (int r = 0; r < M; ++r) {
      double t = 0.0;
#pragma unroll
      for (int k = 0; k < M; ++k) t = fma(K[r * M + k], dj[k], t);
      yj[r] = t;
    }
#pragma unroll 1
    for (int i = 0; i < C; ++i) {
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int q = 0; q < D; ++q)
          t = fma(X[(a * D + q) * C + i] - u[((size_t)nd[a] * C + i) * D + q], yj[a * D + q], t);
      E[i][j] = t;
    }
  }
  const double r = erho[e];
  const double g = p * pow(r, p - 1.0) / ((double)N * N * N);
  double sJ = 0.0;
#pragma unroll
  for (int i = 0; i < C; ++i)
#pragma unroll
    for (int j = 0; j < C; ++j) {
      if (dC) dC[((size_t)lin * C + i) * C + j] = g * E[i][j];
      if (G) sJ = fma(G[i * C + j], E[i][j], sJ);
    }
  if (dJ) dJ[lin] = g * sJ;
}

// Sensitivity filter on the dense periodic grid (x fastest):
// out_e = sum_f H_ef rho_f dc_f / (max(gamma, rho_e) sum_f H_ef), H_ef = max(0, rmin - |x_e - x_f|)
__global__ void k_simp_filter(const double* __restrict__ rho, const double* __restrict__ dc, int N, double rmin,
                              int r, double gamma, double* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t n3 = (size_t)N * N * N;
  if (e >= n3) return;
  const int x = (int)(e % N), y = (int)((e / N) % N), z = (int)(e / ((size_t)N * N));
  double num = 0.0, den = 0.0;
  for (int dz = -r; dz <= r; ++dz)
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx) {
        const double h = rmin - sqrt((double)(dx * dx + dy * dy + dz * dz));
        if (h <= 0.0) continue;
        const size_t f = (size_t)wrapm(x + dx, N) + (size_t)N * (wrapm(y + dy, N) + (size_t)N * wrapm(z + dz, N));
        num += h * rho[f] * dc[f];
        den += h;
      }
  out[e] = num / (fmax(gamma, rho[e]) * den);
}

// OC update of element i for multiplier lam, clipped to the move limit and [lo, 1];
// per-block sums of the updated densities into partial[blockIdx.x]
__global__ __launch_bounds__(kBlock) void k_oc_eval(const double* __restrict__ rho, const double* __restrict__ dc,
                                                    size_t n, double lam, double move, double eta, double lo,
                                                    double* __restrict__ out, double* __restrict__ partial) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock) {
    const double r = rho[i];
    const double B = fmax(-dc[i], 0.0);
    const double cand = r * pow(B / lam, eta);
    const double v = fmin(fmin(1.0, r + move), fmax(cand, fmax(lo, r - move)));
    if (out) out[i] = v;
    acc += v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kBlock / 64; ++k) t += sh[k];
    partial[blockIdx.x] = t;
  }
}

// counter-based uniform(-1,1) values (splitmix64 finaliser of seed + index)
__global__ void k_random(double* __restrict__ x, size_t n, uint64_t seed) {
  size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

inline unsigned blocks_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// One colour of the Gauss-Seidel smoother (Sec. 4.6): u_i += omega D_i^-1 r_i
// for the listed nodes, r the residual of the current iterate at those nodes.
// No two listed nodes share an element, so the updates are independent.
template <typename T>
__global__ void k_gs_update(const int* __restrict__ list, int n_list, int n, int D, const T* __restrict__ dinv,
                            const T* __restrict__ r, T* __restrict__ u, T omega) {
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= (size_t)n_list * D) return;
  const int i = list[t / D];
  const int q = (int)(t % D);
  const size_t idx = vix((int)blockIdx.y, (size_t)n, (size_t)i, D, q);
  u[idx] += omega * dinv[(size_t)i * D + q] * r[idx];
}

// ---------------------------------------------------------------- connected components
// Union-find over the active elements of level 1 with lock-free hooking (the
// scheme of Jaiganesh and Burtscher's ECL-CC): every element points to an
// element of smaller id in its set (parent[v] <= v), a root to itself; a union
// hooks the larger of the two roots under the smaller one by compare-and-swap
// and retries from the value it found when another thread hooked that root
// first.  Ids only decrease along every chain, so each loop ends.
__device__ __forceinline__ int cc_load(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root of v's set, shortening the chain on the way (each element is pointed
// past its parent to its grandparent, which is also in the set)
__device__ int cc_root(int* parent, int v) {
  int cur = cc_load(parent + v);
  if (cur != v) {
    int prev = v, next;
    while (cur > (next = cc_load(parent + cur))) {
      __hip_atomic_store(parent + prev, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      prev = cur;
      cur = next;
    }
  }
  return cur;
}

__global__ void k_cc_init(int* __restrict__ parent, int n_e) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v < n_e) parent[v] = v;
}

// element v is joined to every active element among its 26 periodic
// neighbours (all of them share at least one node with v)
__global__ void k_cc_hook(const int* __restrict__ elem_lin, int n_e, const int* __restrict__ elem_map, int N,
                          int* parent) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n_e) return;
  const int lin = elem_lin[v];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  for (int j = 0; j < 27; ++j) {
    if (j == 13) continue;
    const int w = elem_map[wrapm(x + j % 3 - 1, N) + N * (wrapm(y + (j / 3) % 3 - 1, N) + N * wrapm(z + j / 9 - 1, N))];
    if (w < 0 || w == v) continue;
    int a = cc_root(parent, v), b = cc_root(parent, w);
    while (a != b) {
      if (a < b) {
        const int got = atomicCAS(parent + b, b, a);
        if (got == b) break;
        b = got;  // b was hooked meanwhile: continue from its new parent (smaller)
      } else {
        const int got = atomicCAS(parent + a, a, b);
        if (got == a) break;
        a = got;
      }
    }
  }
}

__global__ void k_cc_count(const int* __restrict__ parent, int n_e, int* __restrict__ count) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  const bool root = v < n_e && parent[v] == v;
  const unsigned long long m = __ballot(root);
  if ((threadIdx.x & 63) == 0 && m) atomicAdd(count, __popcll(m));
}

}  // namespace

// ================================================================ launchers

// coarse-level sweep: CB cases per thread, C / CB grid rows, workgroup size L.bs
template <typename T, int D, int CB, int EPI>
static void launch_coarse(const LevelView<T>& L, int kind, int rows, const T* u, const EpiArgs<T>& e, hipStream_t s) {
  const bool nm = L.cb >= 2;  // neighbour-major variants (64-wide workgroups only)
  const int nrows = L.list ? L.n_list : L.n_n;
  if (nrows <= 0) return;
  if (L.bs == 64 || nm) {
    const dim3 g((unsigned)((nrows + 63) / 64), (unsigned)rows);
    if (kind == KIND_TABLE) {
      if (nm) hipLaunchKernelGGL((k_apply_coarse<T, D, CB, KIND_TABLE, EPI, 64, 1>), g, dim3(64), 0, s, L, u, e);
      else hipLaunchKernelGGL((k_apply_coarse<T, D, CB, KIND_TABLE, EPI, 64>), g, dim3(64), 0, s, L, u, e);
    } else {
      if (nm) hipLaunchKernelGGL((k_apply_coarse<T, D, CB, KIND_PERELEM, EPI, 64, 1>), g, dim3(64), 0, s, L, u, e);
      else hipLaunchKernelGGL((k_apply_coarse<T, D, CB, KIND_PERELEM, EPI, 64>), g, dim3(64), 0, s, L, u, e);
    }
  } else {
    const dim3 g(blocks_for(nrows), (unsigned)rows);
    if (kind == KIND_TABLE)
      hipLaunchKernelGGL((k_apply_coarse<T, D, CB, KIND_TABLE, EPI, kBlock>), g, dim3(kBlock), 0, s, L, u, e);
    else
      hipLaunchKernelGGL((k_apply_coarse<T, D, CB, KIND_PERELEM, EPI, kBlock>), g, dim3(kBlock), 0, s, L, u, e);
  }
}

// staged interior sweep (variant 9): the staged workgroups, then the plain
// kernel (all 27 neighbours of a case loaded up front) over the rest
template <typename T, int D, int EPI>
static void launch_interior_stage(const LevelView<T>& L, int C, const T* u, const EpiArgs<T>& e, hipStream_t s) {
  if (L.n_st_blk > 0) {
    if (L.st_nodes == 512)
      hipLaunchKernelGGL((k_apply_interior_stage<T, D, EPI, 512>), dim3((unsigned)L.n_st_blk), dim3(512), 0, s, L, C,
                         u, e);
    else
      hipLaunchKernelGGL((k_apply_interior_stage<T, D, EPI, 256>), dim3((unsigned)L.n_st_blk), dim3(256), 0, s, L, C,
                         u, e);
  }
  if (L.n_st_rest > 0) {
    LevelView<T> R = L;
    R.interior = L.st_rest;
    R.n_int = L.n_st_rest;
    hipLaunchKernelGGL((k_apply_interior<T, D, EPI, 1>), dim3(blocks_for(R.n_int)), dim3(kBlock), 0, s, R, C, u, e);
  }
}

template <typename T, int D, int C, int EPI>
static void apply_dispatch_kind(const LevelView<T>& L, int kind, const T* u, const EpiArgs<T>& e, hipStream_t s) {
  if (kind == KIND_SHARED) {
    if (L.cb >= 5 && L.cb <= 9) {  // boundary as a register-assembled masked stencil
      if (L.n_int > 0) {
        if (L.cb == 9)
          launch_interior_stage<T, D, EPI>(L, C, u, e, s);
        else if (L.cb == 5)
          hipLaunchKernelGGL((k_apply_interior<T, D, EPI>), dim3(blocks_for(L.n_int)), dim3(kBlock), 0, s, L, C, u, e);
        else if (L.cb == 7 || L.cb == 8)
          hipLaunchKernelGGL((k_apply_interior<T, D, EPI, 1>), dim3(blocks_for(L.n_int)), dim3(kBlock), 0, s, L, C, u, e);
        else
          hipLaunchKernelGGL((k_apply_interior_nc<T, D, C, EPI>), dim3(blocks_for(L.n_int)), dim3(kBlock), 0, s, L, u,
                             e);
      }
      if (L.n_bnd > 0) {
        // one case per thread (C workgroups per node block): the assembly is repeated per case,
        // but the live set stays small (with several cases per thread the
        // compiler hoists every neighbour's loads and spills)
        const dim3 g(blocks_for(L.n_bnd) * C);
        if (L.cb == 8)  // all cases per thread: one assembly per node
          hipLaunchKernelGGL((k_apply_boundary_all<T, D, C, EPI>), dim3(blocks_for(L.n_bnd)), dim3(kBlock), 0, s, L,
                             u, e);
        else if (L.cb == 7 || L.cb == 9)
          hipLaunchKernelGGL((k_apply_boundary_cls<T, D, 1, EPI, 1>), g, dim3(kBlock), 0, s, L, u, e, C);
        else
          hipLaunchKernelGGL((k_apply_boundary_cls<T, D, 1, EPI>), g, dim3(kBlock), 0, s, L, u, e, C);
      }
    } else if (L.cb == 0 || L.cb == 2) {  // all cases per neighbour load
      if (L.n_int > 0)
        hipLaunchKernelGGL((k_apply_interior_nc<T, D, C, EPI>), dim3(blocks_for(L.n_int)), dim3(kBlock), 0, s, L, u, e);
      if (L.n_bnd > 0) {
        if (L.cb == 0)  // boundary as a masked stencil
          hipLaunchKernelGGL((k_apply_boundary_st<T, D, C, EPI>), dim3(blocks_for(L.n_bnd)), dim3(kBlock), 0, s, L, u,
                             e);
        else            // boundary element by element
          hipLaunchKernelGGL((k_apply_boundary_nc<T, D, C, EPI>), dim3(blocks_for(L.n_bnd)), dim3(kBlock), 0, s, L, u,
                             e);
      }
    } else {          // one case per pass over the neighbourhood
      if (L.n_int > 0 && L.cb == 3 && L.n_runs > 0)
        hipLaunchKernelGGL((k_apply_interior_run<T, D, EPI>), dim3(blocks_for(L.n_runs)), dim3(kBlock), 0, s, L, C, u,
                           e);
      else if (L.n_int > 0)
        hipLaunchKernelGGL((k_apply_interior<T, D, EPI>), dim3(blocks_for(L.n_int)), dim3(kBlock), 0, s, L, C, u, e);
      if (L.n_bnd > 0)
        hipLaunchKernelGGL((k_apply_boundary<T, D, EPI>), dim3(blocks_for(L.n_bnd)), dim3(kBlock), 0, s, L, C, u, e);
    }
  } else {
    if (L.n_n == 0) return;
    // cb 0 / 2: all cases per thread; cb 1 / 3: one grid row per case (2, 3: neighbour-major)
    if ((L.cb == 1 || L.cb == 3) && C > 1)
      launch_coarse<T, D, 1, EPI>(L, kind, C, u, e, s);
    else
      launch_coarse<T, D, C, EPI>(L, kind, 1, u, e, s);
  }
  GMT_LAUNCH_CHECK();
}

template <typename T, int D, int C>
static void apply_dispatch_epi(const LevelView<T>& L, int kind, int epi, const T* u, const EpiArgs<T>& e,
                               hipStream_t s) {
  switch (epi) {
    case EPI_KU: apply_dispatch_kind<T, D, C, EPI_KU>(L, kind, u, e, s); break;
    case EPI_RESID: apply_dispatch_kind<T, D, C, EPI_RESID>(L, kind, u, e, s); break;
    case EPI_JACOBI: apply_dispatch_kind<T, D, C, EPI_JACOBI>(L, kind, u, e, s); break;
    case EPI_CHEB: apply_dispatch_kind<T, D, C, EPI_CHEB>(L, kind, u, e, s); break;
    default: apply_dispatch_kind<T, D, C, EPI_CHEB0>(L, kind, u, e, s); break;
  }
}

template <typename T>
void launch_apply(const LevelView<T>& L, int kind, int D, int C, int epi, const T* u, const EpiArgs<T>& e,
                  hipStream_t s) {
  if (D == 3 && C == 6) apply_dispatch_epi<T, 3, 6>(L, kind, epi, u, e, s);
  else if (D == 3 && C == 1) apply_dispatch_epi<T, 3, 1>(L, kind, epi, u, e, s);
  else if (D == 1 && C == 3) apply_dispatch_epi<T, 1, 3>(L, kind, epi, u, e, s);
  else if (D == 1 && C == 1) apply_dispatch_epi<T, 1, 1>(L, kind, epi, u, e, s);
  else fail(GMT_E_INVAL, "unsupported (d, c) = (%d, %d)", D, C);
}

template <typename T>
void launch_smooth_zero(int n, int D, int C, const T* f, const T* dinv, T scale, T* out, T* dvec,
                        hipStream_t s) {
  const size_t tot = (size_t)n * C * D;
  if (!tot) return;
  hipLaunchKernelGGL(k_smooth_zero<T>, dim3(blocks_for((size_t)n * D), C), dim3(kBlock), 0, s, n, D, C, f, dinv,
                     scale, out, dvec);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_normalize(const T* src, size_t n, const double* nrm2, T* dst, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_normalize<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, src, nrm2, dst);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_restrict(const LevelView<T>& F, const LevelView<T>& Cv, int Q, int D, const T* rf, T* fc, hipStream_t s) {
  const unsigned g = blocks_for(Cv.n_n);
  if (!g) return;
  if (Q == 18 && D == 3) hipLaunchKernelGGL((k_restrict<T, 18, 3>), dim3(g), dim3(kBlock), 0, s, F, Cv, rf, fc);
  else if (Q == 3 && D == 1) hipLaunchKernelGGL((k_restrict<T, 3, 1>), dim3(g), dim3(kBlock), 0, s, F, Cv, rf, fc);
  else if (Q == 3 && D == 3) hipLaunchKernelGGL((k_restrict<T, 3, 3>), dim3(g), dim3(kBlock), 0, s, F, Cv, rf, fc);
  else if (Q == 1 && D == 1) hipLaunchKernelGGL((k_restrict<T, 1, 1>), dim3(g), dim3(kBlock), 0, s, F, Cv, rf, fc);
  else fail(GMT_E_INVAL, "unsupported (Q, D) = (%d, %d)", Q, D);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_prolong_add(const LevelView<T>& F, const LevelView<T>& Cv, int Q, int D, const T* uc, T* uf, hipStream_t s) {
  const unsigned g = blocks_for(F.n_n);
  if (!g) return;
  if (Q == 18 && D == 3) hipLaunchKernelGGL((k_prolong_add<T, 18, 3>), dim3(g), dim3(kBlock), 0, s, F, Cv, uc, uf);
  else if (Q == 3 && D == 1) hipLaunchKernelGGL((k_prolong_add<T, 3, 1>), dim3(g), dim3(kBlock), 0, s, F, Cv, uc, uf);
  else if (Q == 3 && D == 3) hipLaunchKernelGGL((k_prolong_add<T, 3, 3>), dim3(g), dim3(kBlock), 0, s, F, Cv, uc, uf);
  else if (Q == 1 && D == 1) hipLaunchKernelGGL((k_prolong_add<T, 1, 1>), dim3(g), dim3(kBlock), 0, s, F, Cv, uc, uf);
  else fail(GMT_E_INVAL, "unsupported (Q, D) = (%d, %d)", Q, D);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_coarse_solve(const T* cinv, int cn, int D, int C, const T* f, T* u, hipStream_t s) {
  const unsigned g = (unsigned)((cn + 63) / 64);
  const dim3 b(64 * kCoarseSplit);
  if (C == 6) hipLaunchKernelGGL((k_coarse_solve<T, 6>), dim3(g), b, 0, s, cinv, cn, D, f, u);
  else if (C == 3) hipLaunchKernelGGL((k_coarse_solve<T, 3>), dim3(g), b, 0, s, cinv, cn, D, f, u);
  else if (C == 1) hipLaunchKernelGGL((k_coarse_solve<T, 1>), dim3(g), b, 0, s, cinv, cn, D, f, u);
  else fail(GMT_E_INVAL, "unsupported C=%d", C);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_fill(T* p, size_t n, T v, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
  GMT_LAUNCH_CHECK();
}

template <typename Tin, typename Tout>
void launch_convert(const Tin* a, Tout* b, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL((k_convert<Tin, Tout>), dim3(blocks_for(n)), dim3(kBlock), 0, s, a, b, n);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_copy(const T* a, T* b, size_t n, hipStream_t s) {
  launch_convert<T, T>(a, b, n, s);
}

template <typename T>
void launch_inv(const T* a, T* b, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_inv<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, b, n);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_gs_update(const int* list, int n_list, int n, int D, int C, const T* dinv, const T* r, T* u, T omega,
                      hipStream_t s) {
  if (n_list <= 0) return;
  hipLaunchKernelGGL(k_gs_update<T>, dim3(blocks_for((size_t)n_list * D), C), dim3(kBlock), 0, s, list, n_list, n, D,
                     dinv, r, u, omega);
  GMT_LAUNCH_CHECK();
}

int count_components(const int* elem_lin, int n_e, const int* elem_map, int N, int* parent, int* d_count,
                     hipStream_t s) {
  if (n_e <= 0) return 0;
  const unsigned g = blocks_for(n_e);
  hipLaunchKernelGGL(k_cc_init, dim3(g), dim3(kBlock), 0, s, parent, n_e);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_cc_hook, dim3(g), dim3(kBlock), 0, s, elem_lin, n_e, elem_map, N, parent);
  GMT_LAUNCH_CHECK();
  GMT_HIP(hipMemsetAsync(d_count, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_cc_count, dim3(g), dim3(kBlock), 0, s, parent, n_e, d_count);
  GMT_LAUNCH_CHECK();
  int h = 0;
  GMT_HIP(hipMemcpyAsync(&h, d_count, sizeof(int), hipMemcpyDeviceToHost, s));
  GMT_HIP(hipStreamSynchronize(s));
  return h;
}

static unsigned red_grid(int n) {
  unsigned g = blocks_for((size_t)n);
  if (g > (unsigned)kRedBlocks) g = kRedBlocks;
  return g == 0 ? 1 : g;
}

template <typename T>
void launch_dot(const T* a, const T* b, int n, int C, int D, double* partial, double* out, hipStream_t s) {
  const unsigned g = red_grid(n);
  if (C == 6 && D == 3) hipLaunchKernelGGL((k_dot<T, 6, 3>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else if (C == 1 && D == 3) hipLaunchKernelGGL((k_dot<T, 1, 3>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else if (C == 3 && D == 1) hipLaunchKernelGGL((k_dot<T, 3, 1>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else if (C == 1 && D == 1) hipLaunchKernelGGL((k_dot<T, 1, 1>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else fail(GMT_E_INVAL, "unsupported (c, d)");
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_final, dim3(C), dim3(kBlock), 0, s, partial, (int)g, C, out);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_dot_centered(const T* a, const T* b, const double* sums, double inv_n, int n, int C, int D, double* partial,
                         double* out, hipStream_t s) {
  const unsigned g = red_grid(n);
  if (C == 6 && D == 3)
    hipLaunchKernelGGL((k_dot<T, 6, 3, true>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial, sums, inv_n);
  else if (C == 3 && D == 1)
    hipLaunchKernelGGL((k_dot<T, 3, 1, true>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial, sums, inv_n);
  else
    fail(GMT_E_INVAL, "unsupported (c, d)");
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_final, dim3(C), dim3(kBlock), 0, s, partial, (int)g, C, out);
  GMT_LAUNCH_CHECK();
}

template <typename Ta, typename Tb>
void launch_gram(const Ta* a, const Tb* b, int n, int C, int D, double* partial, double* out, hipStream_t s) {
  const unsigned g = red_grid(n);
  if (C == 6 && D == 3) hipLaunchKernelGGL((k_gram<Ta, Tb, 6, 3>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else if (C == 3 && D == 1) hipLaunchKernelGGL((k_gram<Ta, Tb, 3, 1>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else fail(GMT_E_INVAL, "unsupported (c, d)");
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_final, dim3(C * C), dim3(kBlock), 0, s, partial, (int)g, C * C, out);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_colsum(const T* v, int n, int Q, int D, double* partial, double* sums, hipStream_t s) {
  const unsigned g = red_grid(n);
  if (Q == 18 && D == 3) hipLaunchKernelGGL((k_colsum<T, 18, 3>), dim3(g), dim3(kBlock), 0, s, v, n, partial);
  else if (Q == 3 && D == 1) hipLaunchKernelGGL((k_colsum<T, 3, 1>), dim3(g), dim3(kBlock), 0, s, v, n, partial);
  else fail(GMT_E_INVAL, "unsupported (Q, D) = (%d, %d)", Q, D);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_final, dim3(Q), dim3(kBlock), 0, s, partial, (int)g, Q, sums);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_axpby(T* y, const T* x, T alpha, T beta, size_t n, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_axpby<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, y, x, alpha, beta, n);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_scale_add_comp(T* y, const T* x, T alpha, const double* add, int n, int C, int D, hipStream_t s) {
  const size_t tot = (size_t)n * C * D;
  if (!tot) return;
  hipLaunchKernelGGL(k_scale_add_comp<T>, dim3(blocks_for(tot)), dim3(kBlock), 0, s, y, x, alpha, add, n, D, tot);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_mul_nodewise(T* v, const T* w, int n, int C, int D, int divide, hipStream_t s) {
  const size_t tot = (size_t)n * C * D;
  if (!tot) return;
  hipLaunchKernelGGL(k_mul_nodewise<T>, dim3(blocks_for(tot)), dim3(kBlock), 0, s, v, w, n, D, divide, tot);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_project(T* v, int n, int Q, int D, double* partial, double* sums, hipStream_t s) {
  const unsigned g = red_grid(n);
  if (Q == 18 && D == 3) hipLaunchKernelGGL((k_colsum<T, 18, 3>), dim3(g), dim3(kBlock), 0, s, v, n, partial);
  else if (Q == 3 && D == 1) hipLaunchKernelGGL((k_colsum<T, 3, 1>), dim3(g), dim3(kBlock), 0, s, v, n, partial);
  else if (Q == 3 && D == 3) hipLaunchKernelGGL((k_colsum<T, 3, 3>), dim3(g), dim3(kBlock), 0, s, v, n, partial);
  else if (Q == 1 && D == 1) hipLaunchKernelGGL((k_colsum<T, 1, 1>), dim3(g), dim3(kBlock), 0, s, v, n, partial);
  else fail(GMT_E_INVAL, "unsupported (Q, D) = (%d, %d)", Q, D);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_final, dim3(Q), dim3(kBlock), 0, s, partial, (int)g, Q, sums);
  GMT_LAUNCH_CHECK();
  if (n == 0) return;
  hipLaunchKernelGGL(k_sub_mean<T>, dim3(blocks_for((size_t)n * D), Q / D), dim3(kBlock), 0, s, v, n, D, sums,
                     1.0 / n);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_pcg_update(T* u, T* r, const T* p, const T* q, const double* alpha, int n, int Q, int D,
                       hipStream_t s, const double* qsums, double inv_n) {
  const size_t tot = (size_t)n * Q;
  if (!tot) return;
  const dim3 g(blocks_for((size_t)n * D), Q / D);
  if (D == 3)
    hipLaunchKernelGGL((k_pcg_update<T, 3>), g, dim3(kBlock), 0, s, u, r, p, q, alpha, n, qsums, inv_n);
  else if (D == 1)
    hipLaunchKernelGGL((k_pcg_update<T, 1>), g, dim3(kBlock), 0, s, u, r, p, q, alpha, n, qsums, inv_n);
  else
    fail(GMT_E_INVAL, "unsupported d = %d", D);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_dot_colsum(const T* a, const T* b, int n, int C, int D, double* partial, double* dots, double* sums,
                       hipStream_t s) {
  const unsigned g = red_grid(n);
  if (C == 6 && D == 3) hipLaunchKernelGGL((k_dot_colsum<T, 6, 3>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else if (C == 3 && D == 1) hipLaunchKernelGGL((k_dot_colsum<T, 3, 1>), dim3(g), dim3(kBlock), 0, s, a, b, n, partial);
  else fail(GMT_E_INVAL, "unsupported (c, d)");
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_split, dim3(C + C * D), dim3(kBlock), 0, s, partial, (int)g, C + C * D, C, dots, sums);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_dot2_centered(const T* r, const T* z, const double* sums, double inv_n, int n, int C, int D,
                          double* partial, double* rz, double* rr, hipStream_t s) {
  const unsigned g = red_grid(n);
  if (C == 6 && D == 3)
    hipLaunchKernelGGL((k_dot2_centered<T, 6, 3>), dim3(g), dim3(kBlock), 0, s, r, z, n, sums, inv_n, partial);
  else if (C == 3 && D == 1)
    hipLaunchKernelGGL((k_dot2_centered<T, 3, 1>), dim3(g), dim3(kBlock), 0, s, r, z, n, sums, inv_n, partial);
  else
    fail(GMT_E_INVAL, "unsupported (c, d)");
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_split, dim3(2 * C), dim3(kBlock), 0, s, partial, (int)g, 2 * C, C, rz, rr);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_pcg_direction(T* p, const T* z, const double* beta, int n, int Q, int D, hipStream_t s,
                          const double* sums, double inv_n) {
  const size_t tot = (size_t)n * Q;
  if (!tot) return;
  const dim3 g(blocks_for((size_t)n * D), Q / D);
  if (D == 3)
    hipLaunchKernelGGL((k_pcg_direction<T, 3>), g, dim3(kBlock), 0, s, p, z, beta, n, sums, inv_n);
  else if (D == 1)
    hipLaunchKernelGGL((k_pcg_direction<T, 1>), g, dim3(kBlock), 0, s, p, z, beta, n, sums, inv_n);
  else
    fail(GMT_E_INVAL, "unsupported d = %d", D);
  GMT_LAUNCH_CHECK();
}

template <typename Tin, typename Tout>
void launch_aos_to_soa(const Tin* a, Tout* b, int n, int C, int D, hipStream_t s) {
  const size_t tot = (size_t)n * C * D;
  if (!tot) return;
  hipLaunchKernelGGL((k_aos_to_soa<Tin, Tout>), dim3(blocks_for(tot)), dim3(kBlock), 0, s, a, b, n, C, D);
  GMT_LAUNCH_CHECK();
}

template <typename Tin, typename Tout>
void launch_soa_to_aos(const Tin* a, Tout* b, int n, int C, int D, hipStream_t s) {
  const size_t tot = (size_t)n * C * D;
  if (!tot) return;
  hipLaunchKernelGGL((k_soa_to_aos<Tin, Tout>), dim3(blocks_for(tot)), dim3(kBlock), 0, s, a, b, n, C, D);
  GMT_LAUNCH_CHECK();
}

void launch_pcg_alpha(const double* rz, const double* pq, double* alpha, int C, hipStream_t s, const double* stop) {
  hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(64), 0, s, rz, pq, alpha, C, stop);
  GMT_LAUNCH_CHECK();
}

void launch_pcg_beta(const double* rz_new, double* rz, double* beta, int C, hipStream_t s, const double* stop) {
  hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(64), 0, s, rz_new, rz, beta, C, stop);
  GMT_LAUNCH_CHECK();
}

void launch_pcg_check(const double* rr, int C, double* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_check, dim3(1), dim3(64), 0, s, rr, C, flags);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_gauge_shift(T* u, int n, int Q, int D, T* tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_node<T>, dim3(1), dim3(64), 0, s, u, n, Q, D, tmp);
  GMT_LAUNCH_CHECK();
  const size_t tot = (size_t)n * Q;
  hipLaunchKernelGGL(k_sub_node<T>, dim3(blocks_for(tot)), dim3(kBlock), 0, s, u, tot, n, D, tmp);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_accumulate(double* u, const T* d, size_t n, hipStream_t s, double a) {
  if (!n) return;
  hipLaunchKernelGGL(k_accumulate<T>, dim3(blocks_for(n)), dim3(kBlock), 0, s, u, d, n, a);
  GMT_LAUNCH_CHECK();
}

void launch_voxel_elem_flags(const uint8_t* vox, size_t n, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_voxel_flags, dim3(blocks_for(n)), dim3(kBlock), 0, s, vox, n, flags);
  GMT_LAUNCH_CHECK();
}

void launch_node_flags(const int* emap, int N, int* nflags, hipStream_t s) {
  const size_t n = (size_t)N * N * N;
  hipLaunchKernelGGL(k_node_flags, dim3(blocks_for(n)), dim3(kBlock), 0, s, emap, N, nflags);
  GMT_LAUNCH_CHECK();
}

void launch_coarsen_flags(const int* femap, int Nf, int* cflags, uint8_t* dcmask, hipStream_t s) {
  const size_t Nc = Nf / 2;
  const size_t n = Nc * Nc * Nc;
  hipLaunchKernelGGL(k_coarsen, dim3(blocks_for(n)), dim3(kBlock), 0, s, femap, Nf, cflags, dcmask);
  GMT_LAUNCH_CHECK();
}

size_t scan_scratch_ints(size_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

int64_t scan_compact(const int* flags, size_t n, int* map_out, int* lin_out, int* scratch, int* d_total,
                     hipStream_t s) {
  const unsigned nb = (unsigned)((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kBlock), 0, s, flags, n, scratch);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, s, scratch, (int)nb, d_total);
  GMT_LAUNCH_CHECK();
  int total = 0;
  GMT_HIP(hipMemcpyAsync(&total, d_total, sizeof(int), hipMemcpyDeviceToHost, s));
  GMT_HIP(hipStreamSynchronize(s));
  if (map_out) {
    hipLaunchKernelGGL(k_scan_compact, dim3(nb), dim3(kBlock), 0, s, flags, n, scratch, map_out, lin_out);
    GMT_LAUNCH_CHECK();
  }
  return total;
}

void launch_occ8(const int* node_lin, int n_n, const int* emap, int N, uint8_t* occ8, hipStream_t s) {
  if (!n_n) return;
  hipLaunchKernelGGL(k_occ8, dim3(blocks_for(n_n)), dim3(kBlock), 0, s, node_lin, n_n, emap, N, occ8);
  GMT_LAUNCH_CHECK();
}

void launch_boundary_nbrs(const int* boundary, int n_bnd, const int* node_lin, const int* node_map, int N, int* table,
                          hipStream_t s) {
  if (!n_bnd) return;
  hipLaunchKernelGGL(k_boundary_nbrs, dim3(blocks_for(n_bnd)), dim3(kBlock), 0, s, boundary, n_bnd, node_lin, node_map,
                     N, table);
  GMT_LAUNCH_CHECK();
}

void launch_run_flags(const int* interior, int n_int, const int* node_lin, int N, int* flags, hipStream_t s) {
  if (!n_int) return;
  hipLaunchKernelGGL(k_run_flags, dim3(blocks_for(n_int)), dim3(kBlock), 0, s, interior, n_int, node_lin, N, flags);
  GMT_LAUNCH_CHECK();
}

void launch_stage_tables(const int* interior, int n_int, const int* node_lin, const int* node_map, int N, int nb,
                         int pass, const int* blk, int n_blk, int* cnt, const long long* off, int* ids, uint16_t* slot,
                         hipStream_t s) {
  const unsigned grid = pass == 0 ? (unsigned)((n_int + nb - 1) / nb) : (unsigned)n_blk;
  if (!n_int || !grid) return;
  if (nb == 512)
    hipLaunchKernelGGL(k_stage_tables<512>, dim3(grid), dim3(512), 0, s, interior, n_int, node_lin, node_map, N, pass,
                       blk, cnt, off, ids, slot);
  else
    hipLaunchKernelGGL(k_stage_tables<256>, dim3(grid), dim3(256), 0, s, interior, n_int, node_lin, node_map, N, pass,
                       blk, cnt, off, ids, slot);
  GMT_LAUNCH_CHECK();
}

// out = the interior ids of the groups blk[0 .. n_blk) (blockDim.x positions
// each, the last group of the list possibly partial), in that order
__global__ void k_gather_blocks(const int* __restrict__ interior, int n_int, const int* __restrict__ blk,
                                int* __restrict__ out) {
  const int t = blk[blockIdx.x] * (int)blockDim.x + (int)threadIdx.x;
  if (t < n_int) out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = interior[t];
}

void launch_gather_blocks(const int* interior, int n_int, int nb, const int* blk, int n_blk, int* out, hipStream_t s) {
  if (!n_blk) return;
  hipLaunchKernelGGL(k_gather_blocks, dim3(n_blk), dim3(nb), 0, s, interior, n_int, blk, out);
  GMT_LAUNCH_CHECK();
}

void launch_occ_flags(const uint8_t* occ8, int n, int want_full, int* flags, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_occ_flags, dim3(blocks_for(n)), dim3(kBlock), 0, s, occ8, n, want_full, flags);
  GMT_LAUNCH_CHECK();
}

void launch_gather_cmask(const int* elem_lin, int n_e, const uint8_t* dense, uint8_t* cmask, hipStream_t s) {
  if (!n_e) return;
  hipLaunchKernelGGL(k_gather_cmask, dim3(blocks_for(n_e)), dim3(kBlock), 0, s, elem_lin, n_e, dense, cmask);
  GMT_LAUNCH_CHECK();
}

void launch_elem_nodes(const int* elem_lin, int n_e, const int* node_map, int N, int* out, hipStream_t s) {
  if (!n_e) return;
  hipLaunchKernelGGL(k_elem_nodes, dim3(blocks_for(n_e)), dim3(kBlock), 0, s, elem_lin, n_e, node_map, N, out);
  GMT_LAUNCH_CHECK();
}

void launch_prol_maps(const int* node_lin, int n_n, int Nf, const int* cmap, int Nc, int* idx, double* w,
                      hipStream_t s) {
  if (!n_n) return;
  hipLaunchKernelGGL(k_prol_maps, dim3(blocks_for(n_n)), dim3(kBlock), 0, s, node_lin, n_n, Nf, cmap, Nc, idx, w);
  GMT_LAUNCH_CHECK();
}

void launch_galerkin(const int* elem_lin_c, int n_e_c, int Nc, const int* emap_f, const uint8_t* cmask_f,
                     const double* Ksrc, int src_kind, int D, const double* Ps, const double* fscale, double* out64,
                     float* out32, hipStream_t s) {
  if (!n_e_c) return;
  if (D == 3)
    hipLaunchKernelGGL(k_galerkin<3>, dim3(n_e_c), dim3(kBlock), 0, s, elem_lin_c, Nc, emap_f, cmask_f, Ksrc,
                       src_kind, Ps, fscale, out64, out32);
  else
    hipLaunchKernelGGL(k_galerkin<1>, dim3(n_e_c), dim3(kBlock), 0, s, elem_lin_c, Nc, emap_f, cmask_f, Ksrc,
                       src_kind, Ps, fscale, out64, out32);
  GMT_LAUNCH_CHECK();
}

template <typename T>
void launch_diagonal(const LevelView<T>& L, int kind, int D, T* diag, hipStream_t s) {
  const unsigned g = blocks_for(L.n_n);
  if (!g) return;
#define GMT_DIAG(DD, KK) hipLaunchKernelGGL((k_diagonal<T, DD, KK>), dim3(g), dim3(kBlock), 0, s, L, diag)
  if (D == 3) {
    if (kind == KIND_SHARED) GMT_DIAG(3, KIND_SHARED);
    else if (kind == KIND_TABLE) GMT_DIAG(3, KIND_TABLE);
    else GMT_DIAG(3, KIND_PERELEM);
  } else {
    if (kind == KIND_SHARED) GMT_DIAG(1, KIND_SHARED);
    else if (kind == KIND_TABLE) GMT_DIAG(1, KIND_TABLE);
    else GMT_DIAG(1, KIND_PERELEM);
  }
#undef GMT_DIAG
  GMT_LAUNCH_CHECK();
}

void launch_expand_elem_matrices(const LevelView<double>& L, int kind, int n_e, int D, const int* elem_lin,
                                 double* out, hipStream_t s) {
  const size_t tot = (size_t)n_e * 64 * D * D;
  if (!tot) return;
  const unsigned g = blocks_for(tot);
#define GMT_EXP(DD, KK) hipLaunchKernelGGL((k_expand_elem<DD, KK>), dim3(g), dim3(kBlock), 0, s, L, n_e, elem_lin, out)
  if (D == 3) {
    if (kind == KIND_SHARED) GMT_EXP(3, KIND_SHARED);
    else if (kind == KIND_TABLE) GMT_EXP(3, KIND_TABLE);
    else GMT_EXP(3, KIND_PERELEM);
  } else {
    if (kind == KIND_SHARED) GMT_EXP(1, KIND_SHARED);
    else if (kind == KIND_TABLE) GMT_EXP(1, KIND_TABLE);
    else GMT_EXP(1, KIND_PERELEM);
  }
#undef GMT_EXP
  GMT_LAUNCH_CHECK();
}

void launch_load_vector(const int* node_lin, const uint8_t* occ8, const double* oscale, int n_n, int D, int C,
                        const double* fe, double* f, hipStream_t s) {
  if (!n_n) return;
  hipLaunchKernelGGL(k_load_vector, dim3(blocks_for(n_n)), dim3(kBlock), 0, s, node_lin, occ8, oscale, n_n, D, C,
                     fe, f);
  GMT_LAUNCH_CHECK();
}

void launch_density_flags(const double* rho, size_t n, double prune, uint8_t* vox, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_density_flags, dim3(blocks_for(n)), dim3(kBlock), 0, s, rho, n, prune, vox);
  GMT_LAUNCH_CHECK();
}

void launch_element_scale(const int* elem_lin, int n_e, const double* rho, double p, double rho_min, double* erho,
                          double* escale, hipStream_t s) {
  if (!n_e) return;
  hipLaunchKernelGGL(k_element_scale, dim3(blocks_for(n_e)), dim3(kBlock), 0, s, elem_lin, n_e, rho, p, rho_min, erho,
                     escale);
  GMT_LAUNCH_CHECK();
}

void launch_node_oscale(const int* node_lin, int n_n, const int* elem_map, int N, const double* escale, double* o64,
                        float* o32, hipStream_t s) {
  if (!n_n) return;
  hipLaunchKernelGGL(k_node_oscale, dim3(blocks_for(n_n)), dim3(kBlock), 0, s, node_lin, n_n, elem_map, N, escale,
                     o64, o32);
  GMT_LAUNCH_CHECK();
}

void launch_iota(int* a, int n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(n)), dim3(kBlock), 0, s, a, n);
  GMT_LAUNCH_CHECK();
}

void launch_simp_sensitivity(const int* elem_lin, int n_e, const int* node_map, int N, int D, int C, const double* u,
                             const double* Ke, const double* X0, const double* erho, double p, const double* G,
                             double* dJ, double* dC, hipStream_t s) {
  if (!n_e) return;
  const unsigned g = blocks_for(n_e);
  if (D == 3 && C == 6)
    hipLaunchKernelGGL((k_simp_sensitivity<3, 6>), dim3(g), dim3(kBlock), 0, s, elem_lin, n_e, node_map, N, u, Ke, X0,
                       erho, p, G, dJ, dC);
  else if (D == 1 && C == 3)
    hipLaunchKernelGGL((k_simp_sensitivity<1, 3>), dim3(g), dim3(kBlock), 0, s, elem_lin, n_e, node_map, N, u, Ke, X0,
                       erho, p, G, dJ, dC);
  else
    fail(GMT_E_INVAL, "sensitivity for (d, c) = (%d, %d) not instantiated", D, C);
  GMT_LAUNCH_CHECK();
}

void launch_simp_filter(const double* rho, const double* dc, int N, double rmin, double gamma, double* out,
                        hipStream_t s) {
  const size_t n3 = (size_t)N * N * N;
  if (!n3) return;
  const int r = (int)std::ceil(rmin) - 1;
  hipLaunchKernelGGL(k_simp_filter, dim3(blocks_for(n3)), dim3(kBlock), 0, s, rho, dc, N, rmin, r, gamma, out);
  GMT_LAUNCH_CHECK();
}

void launch_oc_eval(const double* rho, const double* dc, size_t n, double lam, double move, double eta, double lo,
                    double* out, double* partial, double* total, hipStream_t s) {
  if (!n) return;
  const unsigned g = std::min<unsigned>(kRedBlocks, blocks_for(n));
  hipLaunchKernelGGL(k_oc_eval, dim3(g), dim3(kBlock), 0, s, rho, dc, n, lam, move, eta, lo, out, partial);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kBlock), 0, s, partial, (int)g, 1, total);
  GMT_LAUNCH_CHECK();
}

void launch_random(double* x, size_t n, uint64_t seed, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_random, dim3(blocks_for(n)), dim3(kBlock), 0, s, x, n, seed);
  GMT_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- explicit instantiations

#define GMT_INST_T(T)                                                                                          \
  template void launch_apply<T>(const LevelView<T>&, int, int, int, int, const T*, const EpiArgs<T>&,         \
                                hipStream_t);                                                                \
  template void launch_smooth_zero<T>(int, int, int, const T*, const T*, T, T*, T*, hipStream_t);            \
  template void launch_restrict<T>(const LevelView<T>&, const LevelView<T>&, int, int, const T*, T*,         \
                                   hipStream_t);                                                              \
  template void launch_prolong_add<T>(const LevelView<T>&, const LevelView<T>&, int, int, const T*, T*,      \
                                      hipStream_t);                                                          \
  template void launch_coarse_solve<T>(const T*, int, int, int, const T*, T*, hipStream_t);                  \
  template void launch_fill<T>(T*, size_t, T, hipStream_t);                                                  \
  template void launch_copy<T>(const T*, T*, size_t, hipStream_t);                                           \
  template void launch_inv<T>(const T*, T*, size_t, hipStream_t);                                            \
  template void launch_dot<T>(const T*, const T*, int, int, int, double*, double*, hipStream_t);             \
  template void launch_normalize<T>(const T*, size_t, const double*, T*, hipStream_t);                     \
  template void launch_pcg_update<T>(T*, T*, const T*, const T*, const double*, int, int, int, hipStream_t,     \
                                     const double*, double);                                                   \
  template void launch_dot_colsum<T>(const T*, const T*, int, int, int, double*, double*, double*, hipStream_t); \
  template void launch_dot2_centered<T>(const T*, const T*, const double*, double, int, int, int, double*, double*, \
                                        double*, hipStream_t);                                                 \
  template void launch_pcg_direction<T>(T*, const T*, const double*, int, int, int, hipStream_t, const double*, \
                                        double);                                                               \
  template void launch_dot_centered<T>(const T*, const T*, const double*, double, int, int, int, double*, double*, \
                                       hipStream_t);                                                           \
  template void launch_aos_to_soa<T, T>(const T*, T*, int, int, int, hipStream_t);                           \
  template void launch_soa_to_aos<T, T>(const T*, T*, int, int, int, hipStream_t);                           \
  template void launch_gauge_shift<T>(T*, int, int, int, T*, hipStream_t);                                   \
  template void launch_project<T>(T*, int, int, int, double*, double*, hipStream_t);                          \
  template void launch_colsum<T>(const T*, int, int, int, double*, double*, hipStream_t);                     \
  template void launch_axpby<T>(T*, const T*, T, T, size_t, hipStream_t);                                    \
  template void launch_scale_add_comp<T>(T*, const T*, T, const double*, int, int, int, hipStream_t);         \
  template void launch_mul_nodewise<T>(T*, const T*, int, int, int, int, hipStream_t);                        \
  template void launch_accumulate<T>(double*, const T*, size_t, hipStream_t, double);                                \
  template void launch_diagonal<T>(const LevelView<T>&, int, int, T*, hipStream_t);                            \
  template void launch_gs_update<T>(const int*, int, int, int, int, const T*, const T*, T*, T, hipStream_t);

GMT_INST_T(float)
GMT_INST_T(double)
template void launch_convert<double, float>(const double*, float*, size_t, hipStream_t);
template void launch_aos_to_soa<double, float>(const double*, float*, int, int, int, hipStream_t);
template void launch_aos_to_soa<float, double>(const float*, double*, int, int, int, hipStream_t);
template void launch_soa_to_aos<double, float>(const double*, float*, int, int, int, hipStream_t);
template void launch_soa_to_aos<float, double>(const float*, double*, int, int, int, hipStream_t);
template void launch_convert<float, double>(const float*, double*, size_t, hipStream_t);
template void launch_gram<double, double>(const double*, const double*, int, int, int, double*, double*,
                                          hipStream_t);
template void launch_gram<float, double>(const float*, const double*, int, int, int, double*, double*,
                                         hipStream_t);

}  // namespace gmt
