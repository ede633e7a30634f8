// gfx950 kernels and host orchestration of the learned initializer: a sparse
// 3D conv U-Net on the GMG hierarchy (see include/gmt.h, gmt_nn_*).
//
// All layers are "gather convolutions": out[i] = sum_t x[tab[i][t]] W[t] with
// a per-level neighbour table tab (27 periodic neighbours on one level, the 27
// fine nodes 2X + o_t of a coarse node for pooling, or the parents of a fine
// node for unpooling; one identity tap for the pointwise head layers).
// Activations are stored in BF16 (round to nearest even), weights are the BF16
// rounding of the FP32 master weights, every sum is accumulated in FP32.
// The backward pass uses the same gather kernel with transposed per-tap
// weights and the inverse table (mirrored taps on one level, the unpooling
// table for pooling and vice versa), and a node-chunked reduction for the
// weight gradients.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace gmt {

namespace {

constexpr int kB = 256;
constexpr float kSlope = 0.1f;

template <typename T>
using cp = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0;  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename T>
__device__ __forceinline__ float ldf(const T* p);
template <>
__device__ __forceinline__ float ldf<float>(const float* p) {
  return *p;
}
template <>
__device__ __forceinline__ float ldf<uint16_t>(const uint16_t* p) {
  return bf2f(*p);
}

template <typename T>
__device__ __forceinline__ void stf(T* p, float v);
template <>
__device__ __forceinline__ void stf<float>(float* p, float v) {
  *p = v;
}
template <>
__device__ __forceinline__ void stf<uint16_t>(uint16_t* p, float v) {
  *p = f2bf(v);
}

__device__ __forceinline__ int wrapi(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }

enum Flags { F_BIAS = 1, F_SKIP = 2, F_ACT = 4, F_SCALE = 8 };

// out[i][co] = epilogue( sum_t sum_ci x[tab[i][t]][ci] W[t][ci][co] ); a thread
// computes COUT / SPLIT outputs of one node (blockIdx.y picks which), so small
// levels still launch enough threads
template <typename Tin, typename Tout, int CIN, int COUT, int NTAP, int FLAGS, int SPLIT>
__global__ __launch_bounds__(kB) void k_gconv(int n, const int* __restrict__ tab, const Tin* __restrict__ x,
                                               const float* __restrict__ W, const float* __restrict__ b,
                                               const uint16_t* __restrict__ skip, float scale, Tout* __restrict__ y) {
  static_assert(COUT % SPLIT == 0, "output channels split evenly");
  constexpr int CO = COUT / SPLIT;
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int co0 = blockIdx.y * CO;
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = 0.f;
#pragma unroll 1
  for (int t = 0; t < NTAP; ++t) {
    const int src = (NTAP == 1 && tab == nullptr) ? i : tab[(size_t)i * NTAP + t];
    if (src < 0) continue;
    float xin[CIN];
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci) xin[ci] = ldf<Tin>(x + (size_t)src * CIN + ci);
    // wave-uniform weights of tap t through the constant address space (scalar loads)
    const cp<float> Wt = (cp<float>)(W + (size_t)t * CIN * COUT + co0);
#pragma unroll
    for (int ci = 0; ci < CIN; ++ci)
#pragma unroll
      for (int co = 0; co < CO; ++co) acc[co] = fmaf(xin[ci], Wt[ci * COUT + co], acc[co]);
  }
#pragma unroll
  for (int co = 0; co < CO; ++co) {
    float v = acc[co];
    if constexpr (FLAGS & F_BIAS) v += b[co0 + co];
    if constexpr (FLAGS & F_SKIP) v += bf2f(skip[(size_t)i * COUT + co0 + co]);
    if constexpr (FLAGS & F_ACT) v = v > 0.f ? v : kSlope * v;
    if constexpr (FLAGS & F_SCALE) v *= scale;
    stf<Tout>(y + (size_t)i * COUT + co0 + co, v);
  }
}

// ---------------------------------------------------------------- BF16 MFMA gather convolution
// The same layer as k_gconv for BF16 inputs, as a gather-GEMM on the matrix
// cores: D[co][node] = sum_K Wm[co][K] X[K][node], K = (tap, input channel)
// in steps of 32, with v_mfma_f32_16x16x32_bf16 (A = 16 output channels x 32 K
// from the pre-arranged weights, B = 32 K x 16 nodes gathered straight from
// the node-major BF16 activations, one 16-byte load per lane, FP32
// accumulators).  Lane l of a 16x16x32 operand holds row/column l % 16 and the
// 8 consecutive K values 8 (l / 16) .. 8 (l / 16) + 7; the accumulator lane l
// holds column l % 16 (a node) and rows 4 (l / 16) .. + 3 (four consecutive
// output channels, one 8-byte store).  A wave computes 4 x 16 nodes, so each
// weight fragment is loaded once per 64 nodes.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMfmaRows = 4;  // 16-node column blocks per wave

__device__ __forceinline__ f32x4_t mfma16(uint4 a, uint4 b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                 c, 0, 0, 0);
}

template <typename Tout, int CIN, int COUT, int NTAP, int FLAGS>
__global__ __launch_bounds__(kB) void k_gconv_mfma(int n, const int* __restrict__ tab, const uint16_t* __restrict__ x,
                                                    const uint4* __restrict__ Wm, const float* __restrict__ b,
                                                    const uint16_t* __restrict__ skip, float scale,
                                                    Tout* __restrict__ y) {
  static_assert(CIN % 16 == 0, "input rows are read 8 channels per lane");
  constexpr int KS = (NTAP * CIN + 31) / 32;  // K steps (the last one zero-padded)
  constexpr int NCB = (COUT + 15) / 16;       // 16-channel output blocks
  constexpr int R = kMfmaRows;
  const int lane = threadIdx.x & 63, col = lane & 15, kb = lane >> 4;
  const int base = (blockIdx.x * (kB / 64) + (threadIdx.x >> 6)) * (16 * R);
  if (base >= n) return;  // wave-uniform
  f32x4_t acc[R][NCB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[r][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int s = 0; s < KS; ++s) {
    const int K0 = 32 * s + 8 * kb;
    const int t = K0 / CIN, ci0 = K0 % CIN;
    uint4 xv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int node = base + 16 * r + col;
      int src = -1;
      if (node < n && t < NTAP) src = (NTAP == 1 && tab == nullptr) ? node : tab[(size_t)node * NTAP + t];
      xv[r] = src >= 0 ? *reinterpret_cast<const uint4*>(x + (size_t)src * CIN + ci0) : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      const uint4 wv = Wm[(size_t)(s * NCB + c) * 64 + lane];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r][c] = mfma16(wv, xv[r], acc[r][c]);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int node = base + 16 * r + col;
    if (node >= n) continue;
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      const int c0 = 16 * c + 4 * kb;
      if (c0 >= COUT) continue;
      float v[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float w = acc[r][c][j];
        if (c0 + j < COUT) {
          if constexpr (FLAGS & F_BIAS) w += b[c0 + j];
          if constexpr (FLAGS & F_SKIP) w += bf2f(skip[(size_t)node * COUT + c0 + j]);
        }
        if constexpr (FLAGS & F_ACT) w = w > 0.f ? w : kSlope * w;
        if constexpr (FLAGS & F_SCALE) w *= scale;
        v[j] = w;
      }
      Tout* out = y + (size_t)node * COUT + c0;
      if constexpr (COUT % 4 == 0 && sizeof(Tout) == 2) {
        uint2 pk;
        pk.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
        pk.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
        *reinterpret_cast<uint2*>(out) = pk;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c0 + j < COUT) stf<Tout>(out + j, v[j]);
      }
    }
  }
}

// One layer's weights in the A-operand order of k_gconv_mfma:
// Wm[s][cb][lane][j] = W[t][ci][co] (BF16, round to nearest even) with
// co = 16 cb + lane % 16 and t * CIN + ci = 32 s + 8 (lane / 16) + j; zero
// beyond the last tap or output channel.
struct MfmaLayer {
  int src;  // offset of W [NTAP][CIN][COUT] in the flat FP32 parameters
  int dst;  // offset in the arranged BF16 array (a multiple of 512)
  int ntap, cin, cout, ncb;
};

__global__ void k_arrange_mfma(int nlayers, const MfmaLayer* __restrict__ lay, int total, const float* __restrict__ W,
                               uint16_t* __restrict__ Wm) {
  const int e = blockIdx.x * kB + threadIdx.x;
  if (e >= total) return;
  int k = 0;
  while (k + 1 < nlayers && lay[k + 1].dst <= e) ++k;
  const MfmaLayer L = lay[k];
  const int r = e - L.dst;
  const int j = r & 7, lane = (r >> 3) & 63, blk = r >> 9;
  const int cb = blk % L.ncb, s = blk / L.ncb;
  const int co = 16 * cb + (lane & 15);
  const int K = 32 * s + 8 * (lane >> 4) + j;
  const int t = K / L.cin, ci = K % L.cin;
  const float v = (t < L.ntap && co < L.cout) ? W[L.src + ((size_t)t * L.cin + ci) * L.cout + co] : 0.f;
  Wm[e] = f2bf(v);
}

// Weight gradient dW[t][ci][co] += sum_i x[tab[i][t]][ci] g[i][co] on the FP32
// matrix cores (v_mfma_f32_16x16x4_f32, D[ci][co] += sum over 4 nodes): a wave
// owns a contiguous chunk of nodes and TPW taps and keeps every 16x16 (ci, co)
// tile of those taps in accumulators; per step of 4 nodes lane l loads one
// input value (node l / 16, channel l % 16 of a tile: BF16, gathered through
// the table) and one gradient value (node l / 16, output channel l % 16), and
// the matrix core forms the 4-node outer-product sums.  The gradient rows are
// loaded once per step for all TPW taps.  The four waves of a block (four
// consecutive chunks) add their sums in LDS in wave order and the block writes
// partial[block][t][.]; k_reduce_partials then adds the blocks in a fixed
// order (no float atomics: the gradient is the same bit for bit on every run).
constexpr int kWgradWaves = 4;                    // waves (chunks) per block
constexpr int kWgradTargetWaves = 8192;           // waves per launch (8 per SIMD)
constexpr size_t kPartFloats = (size_t)16 << 20;  // partial sums of one layer (64 MiB)

__device__ __forceinline__ f32x4_t mfma4(float a, float b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int CIN, int COUT, int NTAP, int TPW>
__global__ __launch_bounds__(kB) void k_wgrad(int n, const int* __restrict__ tab, const uint16_t* __restrict__ x,
                                               const float* __restrict__ g, float* __restrict__ partial,
                                               int nodes_per_chunk) {
  static_assert(CIN % 16 == 0, "input channels in tiles of 16");
  static_assert(NTAP % TPW == 0, "taps in groups of TPW");
  constexpr int CIT = CIN / 16, COT = (COUT + 15) / 16, TILES = TPW * CIT * COT;
  __shared__ f32x4_t red[TILES][64];
  const int lane = threadIdx.x & 63, col = lane & 15, kq = lane >> 4, wave = threadIdx.x >> 6;
  const int chunk = blockIdx.x * kWgradWaves + wave;
  const int t0 = blockIdx.y * TPW;
  const int beg = (int)min((long long)n, (long long)chunk * nodes_per_chunk);
  const int end = min(n, beg + nodes_per_chunk);
  f32x4_t acc[TPW][CIT][COT];
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
    for (int i = 0; i < CIT; ++i)
#pragma unroll
      for (int j = 0; j < COT; ++j) acc[tt][i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // Every load is unconditional (indices clamped into range, the value selected
  // away afterwards), so a step's loads issue together, and the table entries of
  // the next step are fetched while the current step's rows are in flight.
  int nxt[TPW];
  auto table_row = [&](int base, int* out) {
    const int node = min(base + kq, end - 1);
    if constexpr (NTAP > 1) {
      const int* row = tab + (size_t)node * NTAP + t0;  // multi-tap layers always have a table
#pragma unroll
      for (int tt = 0; tt < TPW; ++tt) out[tt] = row[tt];
    } else {
      out[0] = tab ? tab[node] : node;
    }
  };
  if (beg < end) table_row(beg, nxt);
#pragma unroll 1
  for (int base = beg; base < end; base += 4) {
    const int node = base + kq;
    const bool ok = node < end;
    const int nodec = min(node, end - 1);
    int src[TPW];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt) src[tt] = nxt[tt];
    float b[COT];
#pragma unroll
    for (int j = 0; j < COT; ++j) {
      const int co = 16 * j + col;
      const float v = g[(size_t)nodec * COUT + min(co, COUT - 1)];
      b[j] = (ok && co < COUT) ? v : 0.f;
    }
    float a[TPW][CIT];
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
      for (int i = 0; i < CIT; ++i) {
        const float v = bf2f(x[(size_t)max(src[tt], 0) * CIN + 16 * i + col]);
        a[tt][i] = (ok && src[tt] >= 0) ? v : 0.f;
      }
    if (base + 4 < end) table_row(base + 4, nxt);
#pragma unroll
    for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
      for (int i = 0; i < CIT; ++i)
#pragma unroll
        for (int j = 0; j < COT; ++j) acc[tt][i][j] = mfma4(a[tt][i], b[j], acc[tt][i][j]);
  }
  // the four waves' sums, added in wave order
  for (int w = 0; w < kWgradWaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int tt = 0; tt < TPW; ++tt)
#pragma unroll
        for (int i = 0; i < CIT; ++i)
#pragma unroll
          for (int j = 0; j < COT; ++j) {
            f32x4_t& r = red[(tt * CIT + i) * COT + j][lane];
            r = w == 0 ? acc[tt][i][j] : r + acc[tt][i][j];
          }
    }
    __syncthreads();
  }
  // lane l of a tile holds D[ci = 16 i + 4 (l / 16) + r][co = 16 j + l % 16], r = 0..3
  for (int e = threadIdx.x; e < TILES * 64; e += kB) {
    const int tile = e / 64, ln = e % 64;
    const int tt = tile / (CIT * COT), i = (tile / COT) % CIT, j = tile % COT;
    const int co = 16 * j + (ln & 15);
    if (co >= COUT) continue;
    float* out = partial + ((size_t)blockIdx.x * NTAP + t0 + tt) * CIN * COUT;
    const f32x4_t v = red[tile][ln];
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(size_t)(16 * i + 4 * (ln >> 4) + r) * COUT + co] = v[r];
  }
}

// dst[e] += sum_{c < chunks} partial[c][e]: a block covers 64 elements with four
// streams (chunks c = s, s + 4, ...), added in stream order (deterministic)
__global__ __launch_bounds__(kB) void k_reduce_partials(size_t per, int chunks, const float* __restrict__ partial,
                                                        float* __restrict__ dst) {
  __shared__ float sh[4][64];
  const int lane = threadIdx.x & 63, st = threadIdx.x >> 6;
  const size_t e = (size_t)blockIdx.x * 64 + lane;
  float sum = 0.f;
  if (e < per)
#pragma unroll 4
    for (int c = st; c < chunks; c += 4) sum += partial[(size_t)c * per + e];
  sh[st][lane] = sum;
  __syncthreads();
  if (st == 0 && e < per) dst[e] += ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
}

inline unsigned reduce_blocks(size_t per) { return (unsigned)((per + 63) / 64); }

// Bias gradient db[co] += sum_i g[i][co]: per-block sums (grid-stride over a
// fixed grid) into partial[block][co], then k_reduce_partials.
template <int COUT>
__global__ __launch_bounds__(kB) void k_bgrad(int n, const float* __restrict__ g, float* __restrict__ partial) {
  __shared__ float sh[kB / 64][COUT];
  float acc[COUT];
#pragma unroll
  for (int co = 0; co < COUT; ++co) acc[co] = 0.f;
  for (int i = blockIdx.x * kB + threadIdx.x; i < n; i += gridDim.x * kB)
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] += g[(size_t)i * COUT + co];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int co = 0; co < COUT; ++co) {
    float v = acc[co];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) sh[w][co] = v;
  }
  __syncthreads();
  if (threadIdx.x < COUT) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kB / 64; ++k) s += sh[k][threadIdx.x];
    partial[(size_t)blockIdx.x * COUT + threadIdx.x] = s;
  }
}

// g[i] *= act'(y[i]) from the stored (BF16) activation output
__global__ void k_act_grad(size_t total, float* __restrict__ g, const uint16_t* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < total) g[i] *= bf2f(y[i]) > 0.f ? 1.f : kSlope;
}

__global__ void k_add(size_t total, float* __restrict__ a, const float* __restrict__ b) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < total) a[i] += b[i];
}

__global__ void k_zero(size_t total, float* __restrict__ a) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < total) a[i] = 0.f;
}

__global__ void k_round_bf16(size_t total, const float* __restrict__ a, float* __restrict__ b) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < total) b[i] = bf2f(f2bf(a[i]));
}

// Wt[t'][co][ci] = W[perm(t)][ci][co] with perm(t) = mirror ? NTAP-1-t : t
__global__ void k_transpose_taps(int ntap, int cin, int cout, int mirror, const float* __restrict__ W,
                                 float* __restrict__ Wt) {
  const size_t e = (size_t)blockIdx.x * kB + threadIdx.x;
  const size_t per = (size_t)cin * cout;
  if (e >= (size_t)ntap * per) return;
  const int t = (int)(e / per);
  const int r = (int)(e % per);
  const int co = r / cin, ci = r % cin;  // Wt[t][co][ci]
  const int ts = mirror ? ntap - 1 - t : t;
  Wt[e] = W[(size_t)ts * per + (size_t)ci * cout + co];
}

__global__ void k_embed(int n, const uint8_t* __restrict__ occ8, const float* __restrict__ E, int C,
                        uint16_t* __restrict__ y) {
  const size_t e = (size_t)blockIdx.x * kB + threadIdx.x;
  if (e >= (size_t)n * C) return;
  const size_t i = e / C;
  const int c = (int)(e % C);
  y[e] = f2bf(E[(size_t)occ8[i] * C + c]);
}

// Embedding gradient dE[o][c] += sum of g[i][c] over the nodes i with occupancy o,
// over the nodes sorted by occupancy (stable; built once at setup): block k sums
// chunk k of that list (one occupancy value, at most kEmbedChunk nodes; thread t
// takes channel t % C of every (kB / C)-th node, the kB / C streams are then
// added in stream order) into partial[k][c], and k_embed_reduce adds the chunks
// of each value in order (deterministic).
constexpr int kEmbedChunk = 4096;

struct EmbedChunk {
  int value, start, count;
};

__global__ __launch_bounds__(kB) void k_embed_grad(const int* __restrict__ nodes, const EmbedChunk* __restrict__ chunks,
                                                   int C, const float* __restrict__ g, float* __restrict__ partial) {
  __shared__ float sh[kB];
  const EmbedChunk ck = chunks[blockIdx.x];
  const int S = kB / C, c = threadIdx.x % C, st = threadIdx.x / C;
  float acc = 0.f;
  if (st < S)
    for (int k = st; k < ck.count; k += S) acc += g[(size_t)nodes[ck.start + k] * C + c];
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < C) {
    float sum = 0.f;
    for (int j = 0; j < S; ++j) sum += sh[j * C + threadIdx.x];
    partial[(size_t)blockIdx.x * C + threadIdx.x] = sum;
  }
}

__global__ void k_embed_reduce(const int* __restrict__ first, int C, const float* __restrict__ partial,
                               float* __restrict__ dE) {
  const int e = blockIdx.x * kB + threadIdx.x;
  if (e >= 256 * C) return;
  const int v = e / C, c = e % C;
  float sum = 0.f;
  for (int k = first[v]; k < first[v + 1]; ++k) sum += partial[(size_t)k * C + c];
  dE[e] += sum;
}

// tables ----------------------------------------------------------------------

// tab[i][t] = id of node x_i + o_t on the same level (periodic), -1 if inactive
__global__ void k_conv_table(int n, const int* __restrict__ node_lin, const int* __restrict__ map, int N,
                             int* __restrict__ tab) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const int lin = node_lin[i];
  const int x = lin % N, y = (lin / N) % N, z = lin / (N * N);
  for (int t = 0; t < 27; ++t) {
    const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
    tab[(size_t)i * 27 + t] = map[wrapi(x + ox, N) + N * (wrapi(y + oy, N) + N * wrapi(z + oz, N))];
  }
}

// coarse node X: tab[X][t] = fine node 2X + o_t (periodic), -1 if inactive
__global__ void k_pool_table(int nc, const int* __restrict__ cnode_lin, int Nc, const int* __restrict__ fmap,
                             int* __restrict__ tab) {
  const int X = blockIdx.x * kB + threadIdx.x;
  if (X >= nc) return;
  const int Nf = 2 * Nc;
  const int lin = cnode_lin[X];
  const int x = lin % Nc, y = (lin / Nc) % Nc, z = lin / (Nc * Nc);
  for (int t = 0; t < 27; ++t) {
    const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
    tab[(size_t)X * 27 + t] =
        fmap[wrapi(2 * x + ox, Nf) + Nf * (wrapi(2 * y + oy, Nf) + Nf * wrapi(2 * z + oz, Nf))];
  }
}

// fine node i: tab[i][t] = coarse X with 2X + o_t = x_i (periodic), -1 if none
__global__ void k_unpool_table(int nf, const int* __restrict__ fnode_lin, int Nf, const int* __restrict__ cmap,
                               int* __restrict__ tab) {
  const int i = blockIdx.x * kB + threadIdx.x;
  if (i >= nf) return;
  const int Nc = Nf / 2;
  const int lin = fnode_lin[i];
  const int x = lin % Nf, y = (lin / Nf) % Nf, z = lin / (Nf * Nf);
  for (int t = 0; t < 27; ++t) {
    const int px = wrapi(x - (t % 3 - 1), Nf), py = wrapi(y - ((t / 3) % 3 - 1), Nf), pz = wrapi(z - (t / 9 - 1), Nf);
    int id = -1;
    if (!(px & 1) && !(py & 1) && !(pz & 1)) id = cmap[(px >> 1) + Nc * ((py >> 1) + Nc * (pz >> 1))];
    tab[(size_t)i * 27 + t] = id;
  }
}

// AdamW on the FP32 master weights (decoupled weight decay on every parameter)
__global__ void k_adamw(size_t total, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, float lr, float b1, float b2, float eps, float wd, float c1, float c2,
                        float gscale) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i >= total) return;
  const float gi = g[i] * gscale;
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] = p[i] * (1.f - lr * wd) - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ __launch_bounds__(kB) void k_norm2(const float* __restrict__ x, size_t n, double* __restrict__ partial) {
  __shared__ double sh[kB / 64];
  double v = 0.0;
  for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB) v += (double)x[i] * x[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < kB / 64; ++k) s += sh[k];
    partial[blockIdx.x] = s;
  }
}

// Column sums of a node-major [n][Q] FP32 array: per-block FP64 partials
// (fixed grid, deterministic order), then one block sums them into the means.
constexpr int kColBlocks = 128;
template <int Q>
__global__ __launch_bounds__(kB) void k_colsum_rows(int n, const float* __restrict__ x, double* __restrict__ partial) {
  __shared__ double sh[kB / 64][Q];
  double acc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) acc[q] = 0.0;
  for (int i = blockIdx.x * kB + threadIdx.x; i < n; i += gridDim.x * kB)
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] += x[(size_t)i * Q + q];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    double v = acc[q];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) sh[w][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < Q) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kB / 64; ++k) t += sh[k][threadIdx.x];
    partial[(size_t)blockIdx.x * Q + threadIdx.x] = t;
  }
}

// supervised term: with t the centred target (t - column mean), per block the FP64
// sums of t^2 and (p - t)^2 (fixed grid, added on the host in block order)
template <int Q>
__global__ __launch_bounds__(kB) void k_sup_sums(int n, const float* __restrict__ p, const float* __restrict__ t,
                                                 const double* __restrict__ mean, double* __restrict__ partial) {
  __shared__ double sh[2][kB / 64];
  double st = 0.0, se = 0.0;
  for (size_t e = (size_t)blockIdx.x * kB + threadIdx.x; e < (size_t)n * Q; e += (size_t)gridDim.x * kB) {
    const double tc = (double)t[e] - mean[e % Q];
    const double d = (double)p[e] - tc;
    st += tc * tc;
    se += d * d;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    st += __shfl_down(st, o, 64);
    se += __shfl_down(se, o, 64);
  }
  if (lane == 0) {
    sh[0][w] = st;
    sh[1][w] = se;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double v = 0.0;
    for (int k = 0; k < kB / 64; ++k) v += sh[threadIdx.x][k];
    partial[(size_t)blockIdx.x * 2 + threadIdx.x] = v;
  }
}

// g += scale (p - (t - mean))
__global__ void k_sup_grad(size_t total, int Q, const float* __restrict__ p, const float* __restrict__ t,
                           const double* __restrict__ mean, float scale, float* __restrict__ g) {
  const size_t e = (size_t)blockIdx.x * kB + threadIdx.x;
  if (e >= total) return;
  g[e] += scale * (float)((double)p[e] - ((double)t[e] - mean[e % Q]));
}

__global__ void k_colmean_final(const double* __restrict__ partial, int nblk, int Q, int n, double* __restrict__ mean) {
  const int q = threadIdx.x;
  if (q >= Q) return;
  double t = 0.0;
  for (int b = 0; b < nblk; ++b) t += partial[(size_t)b * Q + q];
  mean[q] = n > 0 ? t / n : 0.0;
}

__global__ void k_sub_colmean(size_t total, int Q, float* __restrict__ x, const double* __restrict__ mean) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < total) x[i] = (float)((double)x[i] - mean[i % Q]);
}

__global__ void k_ema(float* __restrict__ e, const float* __restrict__ x, size_t n, float decay) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) e[i] = decay * e[i] + (1.f - decay) * x[i];
}

inline unsigned nblk(size_t n) { return (unsigned)((n + kB - 1) / kB); }

}  // namespace

// ============================================================================ launchers

template <typename Tin, typename Tout, int FLAGS>
static void gconv_dispatch(int cin, int cout, int ntap, int n, const int* tab, const void* x, const float* W,
                           const float* b, const uint16_t* skip, float scale, void* y, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = nblk(n);
  // below ~1000 blocks of nodes, a thread per 16 output channels
  const bool split = g < 1024;
#define GC(CI, CO, NT)                                                                                        \
  if (cin == CI && cout == CO && ntap == NT) {                                                               \
    constexpr int SP = CO % 16 == 0 ? CO / 16 : 1;                                                           \
    if (split && SP > 1)                                                                                     \
      hipLaunchKernelGGL((k_gconv<Tin, Tout, CI, CO, NT, FLAGS, SP>), dim3(g, SP), dim3(kB), 0, s, n, tab,    \
                         (const Tin*)x, W, b, skip, scale, (Tout*)y);                                        \
    else                                                                                                     \
      hipLaunchKernelGGL((k_gconv<Tin, Tout, CI, CO, NT, FLAGS, 1>), dim3(g), dim3(kB), 0, s, n, tab,         \
                         (const Tin*)x, W, b, skip, scale, (Tout*)y);                                        \
    GMT_LAUNCH_CHECK();                                                                                      \
    return;                                                                                                  \
  }
  GC(16, 16, 27) GC(32, 32, 27) GC(64, 64, 27) GC(16, 32, 27) GC(32, 64, 27) GC(32, 16, 27) GC(64, 32, 27)
  GC(16, 32, 1) GC(32, 32, 1) GC(64, 32, 1) GC(32, 18, 1) GC(32, 3, 1)
  GC(32, 16, 1) GC(32, 64, 1) GC(18, 32, 1) GC(3, 32, 1) GC(16, 16, 1) GC(64, 64, 1)
#undef GC
  fail(GMT_E_INVAL, "gather conv (%d -> %d, %d taps) not instantiated", cin, cout, ntap);
}

// BF16-input layers of the forward on the matrix cores
template <typename Tout, int FLAGS>
static void mfma_dispatch(int cin, int cout, int ntap, int n, const int* tab, const uint16_t* x, const uint16_t* Wm,
                          const float* b, const uint16_t* skip, float scale, Tout* y, hipStream_t s) {
  if (n <= 0) return;
  const int per_block = (kB / 64) * 16 * kMfmaRows;
  const unsigned g = (unsigned)((n + per_block - 1) / per_block);
  const uint4* w = reinterpret_cast<const uint4*>(Wm);
#define GM(CI, CO, NT)                                                                                              \
  if (cin == CI && cout == CO && ntap == NT) {                                                                     \
    hipLaunchKernelGGL((k_gconv_mfma<Tout, CI, CO, NT, FLAGS>), dim3(g), dim3(kB), 0, s, n, tab, x, w, b, skip, scale, \
                       y);                                                                                          \
    GMT_LAUNCH_CHECK();                                                                                             \
    return;                                                                                                         \
  }
  if constexpr (sizeof(Tout) == 2) {
    GM(16, 16, 27) GM(32, 32, 27) GM(64, 64, 27) GM(16, 32, 27) GM(32, 64, 27) GM(32, 16, 27) GM(64, 32, 27)
    GM(16, 32, 1) GM(32, 32, 1) GM(64, 32, 1) GM(16, 16, 1) GM(64, 64, 1)
  } else {
    GM(32, 18, 1) GM(32, 3, 1)
  }
#undef GM
  fail(GMT_E_INVAL, "MFMA gather conv (%d -> %d, %d taps) not instantiated", cin, cout, ntap);
}

// taps per wave: as many as keep at most 12 accumulator tiles (48 registers), so
// that several waves per SIMD keep enough gathers in flight
constexpr int wgrad_tpw(int cin, int cout, int ntap) {
  const int tiles = (cin / 16) * ((cout + 15) / 16);
  if (ntap == 1) return 1;
  return tiles * 27 <= 12 ? 27 : tiles * 9 <= 12 ? 9 : tiles * 3 <= 12 ? 3 : 1;
}

static void wgrad_dispatch(int cin, int cout, int ntap, int n, const int* tab, const uint16_t* x, const float* g,
                           float* dW, float* partial, hipStream_t s) {
  if (n <= 0) return;
  const size_t per = (size_t)ntap * cin * cout;
#define WG(CI, CO, NT)                                                                                      \
  if (cin == CI && cout == CO && ntap == NT) {                                                             \
    constexpr int TPW = wgrad_tpw(CI, CO, NT), GROUPS = NT / TPW;                                          \
    /* about kWgradTargetWaves waves of at least 64 nodes, within the partial buffer */                    \
    int chunks = std::max(1, std::min((n + 63) / 64, kWgradTargetWaves / GROUPS));                         \
    int blocks = (chunks + kWgradWaves - 1) / kWgradWaves;                                                 \
    blocks = (int)std::max<size_t>(1, std::min<size_t>(blocks, kPartFloats / per));                        \
    chunks = blocks * kWgradWaves;                                                                          \
    const int npc = (n + chunks - 1) / chunks;                                                              \
    hipLaunchKernelGGL((k_wgrad<CI, CO, NT, TPW>), dim3((unsigned)blocks, (unsigned)GROUPS), dim3(kB), 0, s, n, \
                       tab, x, g, partial, npc);                                                            \
    GMT_LAUNCH_CHECK();                                                                                     \
    hipLaunchKernelGGL(k_reduce_partials, dim3(reduce_blocks(per)), dim3(kB), 0, s, per, blocks, partial, dW); \
    GMT_LAUNCH_CHECK();                                                                                     \
    return;                                                                                                 \
  }
  WG(16, 16, 27) WG(32, 32, 27) WG(64, 64, 27) WG(16, 32, 27) WG(32, 64, 27) WG(32, 16, 27) WG(64, 32, 27)
  WG(16, 32, 1) WG(32, 32, 1) WG(64, 32, 1) WG(32, 18, 1) WG(32, 3, 1) WG(16, 16, 1) WG(64, 64, 1)
#undef WG
  fail(GMT_E_INVAL, "weight gradient (%d -> %d, %d taps) not instantiated", cin, cout, ntap);
}

constexpr int kBgradBlocks = 256;

static void bgrad_dispatch(int cout, int n, const float* g, float* db, float* partial, hipStream_t s) {
  if (n <= 0) return;
  const unsigned grid = std::min<unsigned>(kBgradBlocks, nblk(n));
#define BG(CO)                                                                                   \
  if (cout == CO) {                                                                              \
    hipLaunchKernelGGL(k_bgrad<CO>, dim3(grid), dim3(kB), 0, s, n, g, partial);                  \
    GMT_LAUNCH_CHECK();                                                                          \
    hipLaunchKernelGGL(k_reduce_partials, dim3(reduce_blocks(CO)), dim3(kB), 0, s, (size_t)CO, (int)grid, partial, db); \
    GMT_LAUNCH_CHECK();                                                                          \
    return;                                                                                      \
  }
  BG(16) BG(32) BG(64) BG(18) BG(3)
#undef BG
  fail(GMT_E_INVAL, "bias gradient of width %d not instantiated", cout);
}

// ============================================================================ network

// Parameter layout (flat FP32), in this order; the weight files and the oracle's FP64
// network use the same flat vector:
//   E [256][C0]
//   for l < L:      We_l [27][C_l][C_l], be_l [C_l]
//   for l < L-1:    Wp_l [27][C_l][C_{l+1}], bp_l [C_{l+1}]
//                   Wu_l [27][C_{l+1}][C_l], bu_l [C_l]
//                   Wd_l [27][C_l][C_l],     bd_l [C_l]
//                   W1_l [C_l][H], b1_l [H], W2_l [H][H], b2_l [H], W3_l [H][q], b3_l [q]
//   with attention blocks, then for l < L: Wq_l, Wk_l, Wv_l, Wo_l [C_l][C_l]
struct NetLayout {
  int L = 0, H = 0, q = 0;
  bool att = false;
  int C[GMT_NN_MAX_LEVELS] = {0};
  size_t E = 0, We[GMT_NN_MAX_LEVELS], be[GMT_NN_MAX_LEVELS];
  size_t Wp[GMT_NN_MAX_LEVELS], bp[GMT_NN_MAX_LEVELS], Wu[GMT_NN_MAX_LEVELS], bu[GMT_NN_MAX_LEVELS];
  size_t Wd[GMT_NN_MAX_LEVELS], bd[GMT_NN_MAX_LEVELS];
  size_t W1[GMT_NN_MAX_LEVELS], b1[GMT_NN_MAX_LEVELS], W2[GMT_NN_MAX_LEVELS], b2[GMT_NN_MAX_LEVELS];
  size_t W3[GMT_NN_MAX_LEVELS], b3[GMT_NN_MAX_LEVELS];
  size_t Wq[GMT_NN_MAX_LEVELS], Wk[GMT_NN_MAX_LEVELS], Wv[GMT_NN_MAX_LEVELS], Wo[GMT_NN_MAX_LEVELS];
  size_t total = 0;
};

static NetLayout make_layout(const gmt_nn_config& cfg, int q) {
  NetLayout nl;
  nl.L = cfg.levels;
  nl.H = cfg.head;
  nl.q = q;
  nl.att = cfg.attention != 0;
  for (int l = 0; l < nl.L; ++l) nl.C[l] = cfg.channels[l];
  size_t o = 0;
  auto take = [&](size_t n) {
    const size_t r = o;
    o += n;
    return r;
  };
  const int* C = nl.C;
  nl.E = take((size_t)256 * C[0]);
  for (int l = 0; l < nl.L; ++l) {
    nl.We[l] = take((size_t)27 * C[l] * C[l]);
    nl.be[l] = take(C[l]);
  }
  for (int l = 0; l + 1 < nl.L; ++l) {
    nl.Wp[l] = take((size_t)27 * C[l] * C[l + 1]);
    nl.bp[l] = take(C[l + 1]);
    nl.Wu[l] = take((size_t)27 * C[l + 1] * C[l]);
    nl.bu[l] = take(C[l]);
    nl.Wd[l] = take((size_t)27 * C[l] * C[l]);
    nl.bd[l] = take(C[l]);
    nl.W1[l] = take((size_t)C[l] * nl.H);
    nl.b1[l] = take(nl.H);
    nl.W2[l] = take((size_t)nl.H * nl.H);
    nl.b2[l] = take(nl.H);
    nl.W3[l] = take((size_t)nl.H * q);
    nl.b3[l] = take(q);
  }
  if (nl.att)
    for (int l = 0; l < nl.L; ++l) {
      nl.Wq[l] = take((size_t)C[l] * C[l]);
      nl.Wk[l] = take((size_t)C[l] * C[l]);
      nl.Wv[l] = take((size_t)C[l] * C[l]);
      nl.Wo[l] = take((size_t)C[l] * C[l]);
    }
  nl.total = o;
  return nl;
}

struct NNState {
  NetLayout nl;
  std::vector<int*> conv, pool, unpool;                  // neighbour tables
  std::vector<uint16_t*> h, a, t, d, z1, z2;             // BF16 activations
  float* Wb = nullptr;                                   // BF16-rounded weights (FP32 storage)
  uint16_t* Wm = nullptr;                                // forward weights in the MFMA operand order
  MfmaLayer* mlay = nullptr;                             // their layer table (device)
  int n_mlay = 0, m_total = 0;
  std::map<size_t, int> mdst;                            // parameter offset of a layer -> its Wm offset
  float* Wt = nullptr;                                   // transposed weights of one layer
  float *g0 = nullptr, *g1 = nullptr, *g2 = nullptr;     // FP32 gradient scratch (max n_l * max C)
  double* colred = nullptr;                              // column-mean partials + means
  float* part = nullptr;                                 // per-chunk gradient partial sums
  std::vector<float*> gd;                                // dL/dd_l accumulators
  std::vector<float*> ga;                                // dL/ds_l, then dL/da_l accumulators
  // attention blocks: per level the serialization (order[r] = node, inv[node] = r,
  // ser_lin[r] = linear index), q, k, v and the BF16 attention output in that order,
  // its FP32 value and log-sum-exp (backward), and the block output s (node order)
  std::vector<int*> order, inv, ser_lin;
  std::vector<uint16_t*> q, k, v, o16, sb;
  std::vector<float*> o32, lse;
  float* g3 = nullptr;
  // level-1 nodes sorted by occupancy and the chunk table of the embedding gradient
  int* emb_nodes = nullptr;
  EmbedChunk* emb_chunks = nullptr;
  int* emb_first = nullptr;  // [257]: first chunk of every occupancy value
  int n_emb_chunks = 0;
  // the tensor that leaves level l's encoder: s_l with attention, a_l without
  const uint16_t* out(int l) const { return nl.att ? sb[l] : a[l]; }
};

static NNState& nn_state(Hier& h) {
  if (!h.nn) fail(GMT_E_STATE, "gmt_nn_setup has not been called for this hierarchy");
  return *reinterpret_cast<NNState*>(h.nn);
}

void nn_release(Hier& h) {
  delete reinterpret_cast<NNState*>(h.nn);
  h.nn = nullptr;
}

void nn_setup(Hier& h, const gmt_nn_config& cfg, hipStream_t s) {
  if (h.density) fail(GMT_E_INVAL, "the network takes binary occupancy: not a density hierarchy");
  // the network runs on the finest cfg.levels levels of the hierarchy (all of them, or the
  // top of a deeper hierarchy: a network trained at one resolution on a finer cell)
  if (cfg.levels < 2 || cfg.levels > h.L || cfg.levels > GMT_NN_MAX_LEVELS)
    fail(GMT_E_INVAL, "network levels (%d) must be in 2..min(%d, the hierarchy's %d)", cfg.levels,
         GMT_NN_MAX_LEVELS, h.L);
  for (int l = 0; l < cfg.levels; ++l)
    if (cfg.channels[l] != 16 && cfg.channels[l] != 32 && cfg.channels[l] != 64)
      fail(GMT_E_INVAL, "channels must be 16, 32 or 64");
  if (cfg.head != 32) fail(GMT_E_INVAL, "head width must be 32");
  if (cfg.attention != 0 && cfg.attention != 1) fail(GMT_E_INVAL, "attention must be 0 or 1");
  if (h.nn) nn_release(h);
  NNState* S = new NNState();
  h.nn = S;
  S->nl = make_layout(cfg, h.Q);
  const int L = cfg.levels;
  size_t maxnc = 0;
  S->conv.resize(L);
  S->pool.assign(L, nullptr);
  S->unpool.assign(L, nullptr);
  S->h.resize(L);
  S->a.resize(L);
  S->t.assign(L, nullptr);
  S->d.assign(L, nullptr);
  S->z1.assign(L, nullptr);
  S->z2.assign(L, nullptr);
  S->gd.assign(L, nullptr);
  S->ga.assign(L, nullptr);
  for (int l = 0; l < L; ++l) {
    const LevelData& d = h.lv[l];
    const int C = S->nl.C[l];
    maxnc = std::max(maxnc, (size_t)d.n_n * std::max(C, std::max(S->nl.H, h.Q)));
    S->conv[l] = h.alloc<int>((size_t)d.n_n * 27);
    hipLaunchKernelGGL(k_conv_table, dim3(nblk(d.n_n)), dim3(kB), 0, s, d.n_n, d.node_lin, d.node_map, d.N,
                       S->conv[l]);
    GMT_LAUNCH_CHECK();
    S->h[l] = h.alloc<uint16_t>((size_t)d.n_n * C);
    S->a[l] = h.alloc<uint16_t>((size_t)d.n_n * C);
    S->ga[l] = h.alloc<float>((size_t)d.n_n * C);
    if (l + 1 < L) {
      const LevelData& c = h.lv[l + 1];
      S->pool[l] = h.alloc<int>((size_t)c.n_n * 27);
      hipLaunchKernelGGL(k_pool_table, dim3(nblk(c.n_n)), dim3(kB), 0, s, c.n_n, c.node_lin, c.N, d.node_map,
                         S->pool[l]);
      GMT_LAUNCH_CHECK();
      S->unpool[l] = h.alloc<int>((size_t)d.n_n * 27);
      hipLaunchKernelGGL(k_unpool_table, dim3(nblk(d.n_n)), dim3(kB), 0, s, d.n_n, d.node_lin, d.N, c.node_map,
                         S->unpool[l]);
      GMT_LAUNCH_CHECK();
      S->t[l] = h.alloc<uint16_t>((size_t)d.n_n * C);
      S->d[l] = h.alloc<uint16_t>((size_t)d.n_n * C);
      S->z1[l] = h.alloc<uint16_t>((size_t)d.n_n * S->nl.H);
      S->z2[l] = h.alloc<uint16_t>((size_t)d.n_n * S->nl.H);
    }
    S->gd[l] = h.alloc<float>((size_t)d.n_n * C);
  }
  if (S->nl.att) {
    for (auto* v : {&S->order, &S->inv, &S->ser_lin}) v->assign(L, nullptr);
    for (auto* v : {&S->q, &S->k, &S->v, &S->o16, &S->sb}) v->assign(L, nullptr);
    S->o32.assign(L, nullptr);
    S->lse.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
      const LevelData& d = h.lv[l];
      const size_t nc = (size_t)d.n_n * S->nl.C[l];
      S->order[l] = h.alloc<int>(d.n_n);
      S->inv[l] = h.alloc<int>(d.n_n);
      S->ser_lin[l] = h.alloc<int>(d.n_n);
      attention_serialize(d.node_map, d.N, d.n_n, l % 3, S->order[l], S->inv[l], S->ser_lin[l], s);
      S->q[l] = h.alloc<uint16_t>(nc);
      S->k[l] = h.alloc<uint16_t>(nc);
      S->v[l] = h.alloc<uint16_t>(nc);
      S->o16[l] = h.alloc<uint16_t>(nc);
      S->sb[l] = h.alloc<uint16_t>(nc);
      S->o32[l] = h.alloc<float>(nc);
      S->lse[l] = h.alloc<float>((size_t)d.n_n * (S->nl.C[l] / 8));
    }
  }
  S->Wb = h.alloc<float>(S->nl.total);
  {
    // every forward layer's weights, arranged for k_gconv_mfma (512 BF16 per K step and
    // 16-channel output block)
    const NetLayout& N = S->nl;
    std::vector<MfmaLayer> lay;
    int dst = 0;
    auto add = [&](size_t src, int ntap, int cin, int cout) {
      MfmaLayer m{(int)src, dst, ntap, cin, cout, (cout + 15) / 16};
      S->mdst[src] = dst;
      lay.push_back(m);
      dst += ((ntap * cin + 31) / 32) * m.ncb * 512;
    };
    for (int l = 0; l < L; ++l) {
      add(N.We[l], 27, N.C[l], N.C[l]);
      if (l + 1 < L) {
        add(N.Wp[l], 27, N.C[l], N.C[l + 1]);
        add(N.Wu[l], 27, N.C[l + 1], N.C[l]);
        add(N.Wd[l], 27, N.C[l], N.C[l]);
        add(N.W1[l], 1, N.C[l], N.H);
        add(N.W2[l], 1, N.H, N.H);
        add(N.W3[l], 1, N.H, N.q);
      }
      if (N.att) {
        add(N.Wq[l], 1, N.C[l], N.C[l]);
        add(N.Wk[l], 1, N.C[l], N.C[l]);
        add(N.Wv[l], 1, N.C[l], N.C[l]);
        add(N.Wo[l], 1, N.C[l], N.C[l]);
      }
    }
    S->n_mlay = (int)lay.size();
    S->m_total = dst;
    S->Wm = h.alloc<uint16_t>((size_t)dst);
    S->mlay = h.alloc<MfmaLayer>(lay.size());
    GMT_HIP(hipMemcpyAsync(S->mlay, lay.data(), lay.size() * sizeof(MfmaLayer), hipMemcpyHostToDevice, s));
  }
  size_t maxw = 0;
  for (int l = 0; l < L; ++l) maxw = std::max(maxw, (size_t)27 * 64 * 64);
  S->Wt = h.alloc<float>(maxw);
  S->colred = h.alloc<double>((size_t)(kColBlocks + 1) * 32);
  S->g0 = h.alloc<float>(maxnc);
  S->g1 = h.alloc<float>(maxnc);
  S->g2 = h.alloc<float>(maxnc);
  if (S->nl.att) S->g3 = h.alloc<float>(maxnc);
  S->part = h.alloc<float>(std::max(kPartFloats, (size_t)kBgradBlocks * 64));
  GMT_HIP(hipStreamSynchronize(s));
}

size_t nn_param_count(const gmt_nn_config& cfg, int q) { return make_layout(cfg, q).total; }

// x[n][Q] -= column means over the n rows (the zero-mean gauge of a prediction;
// the same map is its own adjoint, so the backward applies it to the gradient)
static void center_rows(NNState& S, float* x, int n, int Q, hipStream_t s) {
  if (n <= 0) return;
  double* partial = S.colred;
  double* mean = S.colred + (size_t)kColBlocks * 32;
  if (Q == 18)
    hipLaunchKernelGGL(k_colsum_rows<18>, dim3(kColBlocks), dim3(kB), 0, s, n, x, partial);
  else if (Q == 3)
    hipLaunchKernelGGL(k_colsum_rows<3>, dim3(kColBlocks), dim3(kB), 0, s, n, x, partial);
  else
    fail(GMT_E_INVAL, "prediction width %d not instantiated", Q);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_colmean_final, dim3(1), dim3(64), 0, s, partial, kColBlocks, Q, n, mean);
  GMT_LAUNCH_CHECK();
  const size_t tot = (size_t)n * Q;
  hipLaunchKernelGGL(k_sub_colmean, dim3(nblk(tot)), dim3(kB), 0, s, tot, Q, x, mean);
  GMT_LAUNCH_CHECK();
}

// out[l]: level l (0-based, l < L-1) prediction [n_l][q] FP32 (u_hat^1 for l = 0, e_hat^{l+1} otherwise)
void nn_forward(Hier& h, const float* params, float* const* out, hipStream_t s) {
  NNState& S = nn_state(h);
  const NetLayout& N = S.nl;
  const int L = N.L;
  hipLaunchKernelGGL(k_round_bf16, dim3(nblk(N.total)), dim3(kB), 0, s, N.total, params, S.Wb);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_arrange_mfma, dim3(nblk(S.m_total)), dim3(kB), 0, s, S.n_mlay, S.mlay, S.m_total, params,
                     S.Wm);
  GMT_LAUNCH_CHECK();
  const float* W = S.Wb;
  auto wm = [&](size_t src) { return S.Wm + S.mdst.at(src); };
  const int n0 = h.lv[0].n_n;
  hipLaunchKernelGGL(k_embed, dim3(nblk((size_t)n0 * N.C[0])), dim3(kB), 0, s, n0, h.lv[0].occ8, W + N.E, N.C[0],
                     S.h[0]);
  GMT_LAUNCH_CHECK();
  for (int l = 0; l < L; ++l) {
    const int n = h.lv[l].n_n, C = N.C[l];
    mfma_dispatch<uint16_t, F_BIAS | F_ACT>(C, C, 27, n, S.conv[l], S.h[l], wm(N.We[l]), W + N.be[l], nullptr, 1.f,
                                            S.a[l], s);
    if (N.att) {
      // q, k, v computed straight into serialization order (gathered through order),
      // s = a + o Wo back in node order (o gathered through inv)
      mfma_dispatch<uint16_t, 0>(C, C, 1, n, S.order[l], S.a[l], wm(N.Wq[l]), nullptr, nullptr, 1.f, S.q[l], s);
      mfma_dispatch<uint16_t, 0>(C, C, 1, n, S.order[l], S.a[l], wm(N.Wk[l]), nullptr, nullptr, 1.f, S.k[l], s);
      mfma_dispatch<uint16_t, 0>(C, C, 1, n, S.order[l], S.a[l], wm(N.Wv[l]), nullptr, nullptr, 1.f, S.v[l], s);
      attention_forward(n, attention_window(l), C, h.lv[l].N, S.ser_lin[l], S.q[l], S.k[l], S.v[l], S.o32[l],
                        S.o16[l], S.lse[l], s);
      mfma_dispatch<uint16_t, F_SKIP>(C, C, 1, n, S.inv[l], S.o16[l], wm(N.Wo[l]), nullptr, S.a[l], 1.f, S.sb[l], s);
    }
    if (l + 1 < L)
      mfma_dispatch<uint16_t, F_BIAS | F_ACT>(C, N.C[l + 1], 27, h.lv[l + 1].n_n, S.pool[l], S.out(l), wm(N.Wp[l]),
                                              W + N.bp[l], nullptr, 1.f, S.h[l + 1], s);
  }
  for (int l = L - 2; l >= 0; --l) {
    const int n = h.lv[l].n_n, C = N.C[l];
    const uint16_t* dn = l + 1 == L - 1 ? S.out(L - 1) : S.d[l + 1];
    mfma_dispatch<uint16_t, F_BIAS | F_SKIP | F_ACT>(N.C[l + 1], C, 27, n, S.unpool[l], dn, wm(N.Wu[l]), W + N.bu[l],
                                                     S.out(l), 1.f, S.t[l], s);
    mfma_dispatch<uint16_t, F_BIAS | F_ACT>(C, C, 27, n, S.conv[l], S.t[l], wm(N.Wd[l]), W + N.bd[l], nullptr, 1.f,
                                            S.d[l], s);
    mfma_dispatch<uint16_t, F_BIAS | F_ACT>(C, N.H, 1, n, nullptr, S.d[l], wm(N.W1[l]), W + N.b1[l], nullptr, 1.f,
                                            S.z1[l], s);
    mfma_dispatch<uint16_t, F_BIAS | F_ACT>(N.H, N.H, 1, n, nullptr, S.z1[l], wm(N.W2[l]), W + N.b2[l], nullptr, 1.f,
                                            S.z2[l], s);
    if (out[l]) {
      mfma_dispatch<float, F_BIAS | F_SCALE>(N.H, N.q, 1, n, nullptr, S.z2[l], wm(N.W3[l]), W + N.b3[l], nullptr,
                                             (float)h.N, out[l], s);
      center_rows(S, out[l], n, N.q, s);
    }
  }
}

static void transpose_taps(NNState& S, const float* W, int ntap, int cin, int cout, bool mirror, hipStream_t s) {
  const size_t tot = (size_t)ntap * cin * cout;
  hipLaunchKernelGGL(k_transpose_taps, dim3(nblk(tot)), dim3(kB), 0, s, ntap, cin, cout, mirror ? 1 : 0, W, S.Wt);
  GMT_LAUNCH_CHECK();
}

static void act_grad(float* g, const uint16_t* y, size_t tot, hipStream_t s) {
  if (!tot) return;
  hipLaunchKernelGGL(k_act_grad, dim3(nblk(tot)), dim3(kB), 0, s, tot, g, y);
  GMT_LAUNCH_CHECK();
}

static void addv(float* a, const float* b, size_t tot, hipStream_t s) {
  if (!tot) return;
  hipLaunchKernelGGL(k_add, dim3(nblk(tot)), dim3(kB), 0, s, tot, a, b);
  GMT_LAUNCH_CHECK();
}

static void zerov(float* a, size_t tot, hipStream_t s) {
  if (!tot) return;
  hipLaunchKernelGGL(k_zero, dim3(nblk(tot)), dim3(kB), 0, s, tot, a);
  GMT_LAUNCH_CHECK();
}

__global__ void k_scale_copy(size_t total, const float* __restrict__ a, float sc, float* __restrict__ b) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < total) b[i] = sc * a[i];
}

// y = gather-conv of an FP32 gradient with the transposed per-tap weights held in S.Wt
static void dgrad(NNState& S, int cin, int cout, int ntap, int n_out, const int* tab, const float* g, float* y,
                  hipStream_t s) {
  gconv_dispatch<float, float, 0>(cin, cout, ntap, n_out, tab, g, S.Wt, nullptr, nullptr, 1.f, y, s);
}

// Backward of level l's attention block s = a + bf16(Attn(q, k, v)) Wo with q, k, v = a Wq, a Wk,
// a Wv: on entry S.ga[l] holds dL/ds, on return dL/da (the residual path plus the three
// projections); adds the gradients of Wq, Wk, Wv, Wo.
static void attention_block_backward(Hier& h, NNState& S, int l, float* grad, hipStream_t s) {
  const NetLayout& N = S.nl;
  const float* W = S.Wb;
  const int n = h.lv[l].n_n, C = N.C[l];
  const size_t tc = (size_t)n * C;
  float* gs = S.ga[l];
  // Wo: rows are nodes, the input o is gathered through inv
  wgrad_dispatch(C, C, 1, n, S.inv[l], S.o16[l], gs, grad + N.Wo[l], S.part, s);
  transpose_taps(S, W + N.Wo[l], 1, C, C, false, s);
  dgrad(S, C, C, 1, n, S.order[l], gs, S.g0, s);  // dL/do in serialization order
  attention_backward(n, attention_window(l), C, h.lv[l].N, S.ser_lin[l], S.q[l], S.k[l], S.v[l], S.o32[l],
                     S.lse[l], S.g0, S.g1, S.g2, S.g3, s);
  const size_t Wx[3] = {N.Wq[l], N.Wk[l], N.Wv[l]};
  float* gx[3] = {S.g1, S.g2, S.g3};
  for (int j = 0; j < 3; ++j) {
    // rows in serialization order, the input a gathered through order; dL/da += gathered back through inv
    wgrad_dispatch(C, C, 1, n, S.order[l], S.a[l], gx[j], grad + Wx[j], S.part, s);
    transpose_taps(S, W + Wx[j], 1, C, C, false, s);
    dgrad(S, C, C, 1, n, S.inv[l], gx[j], S.g0, s);
    addv(gs, S.g0, tc, s);
  }
}

// The embedding gradient's node order (level-1 nodes grouped by occupancy, stable)
// and its chunk table, built on the first backward (inference never needs it).
static void embed_order(Hier& h, NNState& S, hipStream_t s) {
  if (S.emb_nodes) return;
  const int n0 = h.lv[0].n_n;
  std::vector<uint8_t> occ((size_t)n0);
  GMT_HIP(hipMemcpyAsync(occ.data(), h.lv[0].occ8, (size_t)n0, hipMemcpyDeviceToHost, s));
  GMT_HIP(hipStreamSynchronize(s));
  std::vector<int> cnt(257, 0), nodes((size_t)n0);
  for (int i = 0; i < n0; ++i) ++cnt[occ[i] + 1];
  for (int v = 0; v < 256; ++v) cnt[v + 1] += cnt[v];
  std::vector<int> pos(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < n0; ++i) nodes[pos[occ[i]]++] = i;
  std::vector<EmbedChunk> ch;
  std::vector<int> first(257, 0);
  for (int v = 0; v < 256; ++v) {
    first[v] = (int)ch.size();
    for (int b = cnt[v]; b < cnt[v + 1]; b += kEmbedChunk) ch.push_back({v, b, std::min(kEmbedChunk, cnt[v + 1] - b)});
  }
  first[256] = (int)ch.size();
  S.n_emb_chunks = (int)ch.size();
  S.emb_nodes = h.alloc<int>(std::max(n0, 1));
  S.emb_chunks = h.alloc<EmbedChunk>(std::max<size_t>(ch.size(), 1));
  S.emb_first = h.alloc<int>(257);
  GMT_HIP(hipMemcpyAsync(S.emb_nodes, nodes.data(), (size_t)n0 * sizeof(int), hipMemcpyHostToDevice, s));
  if (!ch.empty())
    GMT_HIP(hipMemcpyAsync(S.emb_chunks, ch.data(), ch.size() * sizeof(EmbedChunk), hipMemcpyHostToDevice, s));
  GMT_HIP(hipMemcpyAsync(S.emb_first, first.data(), 257 * sizeof(int), hipMemcpyHostToDevice, s));
  GMT_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
}

// grad += d/dparams sum_l <gout[l], out[l]> (activations of the last forward)
void nn_backward(Hier& h, const float* const* gout, float* grad, hipStream_t s) {
  NNState& S = nn_state(h);
  const NetLayout& N = S.nl;
  const int L = N.L, H = N.H, q = N.q;
  const float* W = S.Wb;
  for (int l = 0; l < L; ++l) zerov(S.gd[l], (size_t)h.lv[l].n_n * N.C[l], s);
  // heads: out = N (z2 W3 + b3), z2 = act(z1 W2 + b2), z1 = act(d W1 + b1)
  for (int l = 0; l + 1 < L; ++l) {
    if (!gout[l]) continue;
    const int n = h.lv[l].n_n, C = N.C[l];
    const size_t tq = (size_t)n * q;
    hipLaunchKernelGGL(k_scale_copy, dim3(nblk(tq)), dim3(kB), 0, s, tq, gout[l], (float)h.N, S.g2);
    GMT_LAUNCH_CHECK();
    center_rows(S, S.g2, n, q, s);
    wgrad_dispatch(H, q, 1, n, nullptr, S.z2[l], S.g2, grad + N.W3[l], S.part, s);
    bgrad_dispatch(q, n, S.g2, grad + N.b3[l], S.part, s);
    transpose_taps(S, W + N.W3[l], 1, H, q, false, s);
    dgrad(S, q, H, 1, n, nullptr, S.g2, S.g0, s);
    act_grad(S.g0, S.z2[l], (size_t)n * H, s);
    wgrad_dispatch(H, H, 1, n, nullptr, S.z1[l], S.g0, grad + N.W2[l], S.part, s);
    bgrad_dispatch(H, n, S.g0, grad + N.b2[l], S.part, s);
    transpose_taps(S, W + N.W2[l], 1, H, H, false, s);
    dgrad(S, H, H, 1, n, nullptr, S.g0, S.g1, s);
    act_grad(S.g1, S.z1[l], (size_t)n * H, s);
    wgrad_dispatch(C, H, 1, n, nullptr, S.d[l], S.g1, grad + N.W1[l], S.part, s);
    bgrad_dispatch(H, n, S.g1, grad + N.b1[l], S.part, s);
    transpose_taps(S, W + N.W1[l], 1, C, H, false, s);
    dgrad(S, H, C, 1, n, nullptr, S.g1, S.g2, s);
    addv(S.gd[l], S.g2, (size_t)n * C, s);
  }
  // decoder, finest first: d_l = act(conv(t_l) + bd), t_l = act(unpool(d_{l+1}) + bu + a_l)
  for (int l = 0; l + 1 < L; ++l) {
    const int n = h.lv[l].n_n, C = N.C[l], Cn = N.C[l + 1], nn = h.lv[l + 1].n_n;
    const size_t tc = (size_t)n * C;
    GMT_HIP(hipMemcpyAsync(S.g0, S.gd[l], tc * sizeof(float), hipMemcpyDeviceToDevice, s));
    act_grad(S.g0, S.d[l], tc, s);
    wgrad_dispatch(C, C, 27, n, S.conv[l], S.t[l], S.g0, grad + N.Wd[l], S.part, s);
    bgrad_dispatch(C, n, S.g0, grad + N.bd[l], S.part, s);
    transpose_taps(S, W + N.Wd[l], 27, C, C, true, s);
    dgrad(S, C, C, 27, n, S.conv[l], S.g0, S.g1, s);
    act_grad(S.g1, S.t[l], tc, s);
    // skip path into a_l, bias bu
    GMT_HIP(hipMemcpyAsync(S.ga[l], S.g1, tc * sizeof(float), hipMemcpyDeviceToDevice, s));
    bgrad_dispatch(C, n, S.g1, grad + N.bu[l], S.part, s);
    const uint16_t* dn = l + 1 == L - 1 ? S.out(L - 1) : S.d[l + 1];
    wgrad_dispatch(Cn, C, 27, n, S.unpool[l], dn, S.g1, grad + N.Wu[l], S.part, s);
    transpose_taps(S, W + N.Wu[l], 27, Cn, C, false, s);
    dgrad(S, C, Cn, 27, nn, S.pool[l], S.g1, S.g2, s);
    addv(S.gd[l + 1], S.g2, (size_t)nn * Cn, s);
  }
  // s_{L-1} = d_{L-1}
  GMT_HIP(hipMemcpyAsync(S.ga[L - 1], S.gd[L - 1], (size_t)h.lv[L - 1].n_n * N.C[L - 1] * sizeof(float),
                         hipMemcpyDeviceToDevice, s));
  // encoder, coarsest first: a_l = act(conv(h_l) + be), s_l = block(a_l) (or a_l),
  // h_{l+1} = act(pool(s_l) + bp)
  for (int l = L - 1; l >= 0; --l) {
    const int n = h.lv[l].n_n, C = N.C[l];
    const size_t tc = (size_t)n * C;
    if (N.att) attention_block_backward(h, S, l, grad, s);  // ga[l]: dL/ds_l -> dL/da_l
    GMT_HIP(hipMemcpyAsync(S.g0, S.ga[l], tc * sizeof(float), hipMemcpyDeviceToDevice, s));
    act_grad(S.g0, S.a[l], tc, s);
    wgrad_dispatch(C, C, 27, n, S.conv[l], S.h[l], S.g0, grad + N.We[l], S.part, s);
    bgrad_dispatch(C, n, S.g0, grad + N.be[l], S.part, s);
    transpose_taps(S, W + N.We[l], 27, C, C, true, s);
    dgrad(S, C, C, 27, n, S.conv[l], S.g0, S.g1, s);
    if (l > 0) {
      const int Cp = N.C[l - 1], np = h.lv[l - 1].n_n;
      act_grad(S.g1, S.h[l], tc, s);
      wgrad_dispatch(Cp, C, 27, n, S.pool[l - 1], S.out(l - 1), S.g1, grad + N.Wp[l - 1], S.part, s);
      bgrad_dispatch(C, n, S.g1, grad + N.bp[l - 1], S.part, s);
      transpose_taps(S, W + N.Wp[l - 1], 27, Cp, C, false, s);
      dgrad(S, C, Cp, 27, np, S.unpool[l - 1], S.g1, S.g2, s);
      addv(S.ga[l - 1], S.g2, (size_t)np * Cp, s);
    } else {
      embed_order(h, S, s);
      if (S.n_emb_chunks > 0) {
        hipLaunchKernelGGL(k_embed_grad, dim3(S.n_emb_chunks), dim3(kB), 0, s, S.emb_nodes, S.emb_chunks, C, S.g1,
                           S.part);
        GMT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_embed_reduce, dim3(nblk((size_t)256 * C)), dim3(kB), 0, s, S.emb_first, C, S.part,
                           grad + N.E);
        GMT_LAUNCH_CHECK();
      }
    }
  }
}

__global__ void k_widen(size_t total, const uint16_t* __restrict__ a, float* __restrict__ b) {
  const size_t i = (size_t)blockIdx.x * kB + threadIdx.x;
  if (i < total) b[i] = bf2f(a[i]);
}

// Supervised term on the level-1 prediction p [n][Q] against a solution target t
// (centred here, as p is): loss = alpha |p - t_c|^2 / |t_c|^2, grad += its gradient.
double nn_supervised(Hier& h, const float* p, const float* t, double alpha, float* grad, hipStream_t s) {
  NNState& S = nn_state(h);
  const int n = h.lv[0].n_n, Q = S.nl.q;
  if (n <= 0) return 0.0;
  double* partial = S.colred;
  double* mean = S.colred + (size_t)kColBlocks * 32;
  if (Q == 18)
    hipLaunchKernelGGL(k_colsum_rows<18>, dim3(kColBlocks), dim3(kB), 0, s, n, t, partial);
  else
    hipLaunchKernelGGL(k_colsum_rows<3>, dim3(kColBlocks), dim3(kB), 0, s, n, t, partial);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_colmean_final, dim3(1), dim3(64), 0, s, partial, kColBlocks, Q, n, mean);
  GMT_LAUNCH_CHECK();
  // the sums reuse the front of the partial buffer (the column sums are consumed)
  if (Q == 18)
    hipLaunchKernelGGL(k_sup_sums<18>, dim3(kColBlocks), dim3(kB), 0, s, n, p, t, mean, partial);
  else
    hipLaunchKernelGGL(k_sup_sums<3>, dim3(kColBlocks), dim3(kB), 0, s, n, p, t, mean, partial);
  GMT_LAUNCH_CHECK();
  std::vector<double> hp((size_t)kColBlocks * 2);
  GMT_HIP(hipMemcpyAsync(hp.data(), partial, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  GMT_HIP(hipStreamSynchronize(s));
  double st = 0.0, se = 0.0;
  for (int b = 0; b < kColBlocks; ++b) {
    st += hp[(size_t)2 * b];
    se += hp[(size_t)2 * b + 1];
  }
  if (!(st > 0.0)) fail(GMT_E_INVAL, "the supervised target is zero after centring");
  if (grad) {
    const size_t tot = (size_t)n * Q;
    hipLaunchKernelGGL(k_sup_grad, dim3(nblk(tot)), dim3(kB), 0, s, tot, Q, p, t, mean, (float)(2.0 * alpha / st),
                       grad);
    GMT_LAUNCH_CHECK();
  }
  return alpha * se / st;
}

double nn_time_attention(Hier& h, int l, int reps, hipStream_t s) {
  NNState& S = nn_state(h);
  if (!S.nl.att) fail(GMT_E_STATE, "the network was set up without attention blocks");
  if (l >= S.nl.L) fail(GMT_E_INVAL, "level %d is below the network's %d levels", l + 1, S.nl.L);
  const int n = h.lv[l].n_n, C = S.nl.C[l];
  auto run = [&] {
    attention_forward(n, attention_window(l), C, h.lv[l].N, S.ser_lin[l], S.q[l], S.k[l], S.v[l], S.o32[l],
                      S.o16[l], S.lse[l], s);
  };
  run();  // warm
  hipEvent_t e0, e1;
  GMT_HIP(hipEventCreate(&e0));
  GMT_HIP(hipEventCreate(&e1));
  GMT_HIP(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r) run();
  GMT_HIP(hipEventRecord(e1, s));
  GMT_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  GMT_HIP(hipEventElapsedTime(&ms, e0, e1));
  GMT_HIP(hipEventDestroy(e0));
  GMT_HIP(hipEventDestroy(e1));
  return (double)ms / reps;
}

void nn_serialization(Hier& h, int l, int* out, hipStream_t s) {
  NNState& S = nn_state(h);
  if (!S.nl.att) fail(GMT_E_STATE, "the network was set up without attention blocks");
  if (l >= S.nl.L) fail(GMT_E_INVAL, "level %d is below the network's %d levels", l + 1, S.nl.L);
  GMT_HIP(hipMemcpyAsync(out, S.order[l], (size_t)h.lv[l].n_n * sizeof(int), hipMemcpyDeviceToDevice, s));
}

int nn_activation(Hier& h, int l, int which, float* out, hipStream_t s) {
  NNState& S = nn_state(h);
  const NetLayout& N = S.nl;
  if (which < 0 || which > 10) fail(GMT_E_INVAL, "activation kind %d outside 0..10", which);
  if (which >= 7 && !N.att) fail(GMT_E_STATE, "activation kind %d exists with attention blocks only", which);
  if (l >= N.L) fail(GMT_E_INVAL, "level %d is below the network's %d levels", l + 1, N.L);
  if (which >= 2 && which <= 5 && l >= N.L - 1)
    fail(GMT_E_INVAL, "decoder/head activations exist below the coarsest level only");
  const int width = which == 4 || which == 5 ? N.H : N.C[l];
  if (which == 10) {
    if (out) GMT_HIP(hipMemcpyAsync(out, S.o32[l], (size_t)h.lv[l].n_n * width * sizeof(float),
                                    hipMemcpyDeviceToDevice, s));
    return width;
  }
  const uint16_t* src = which == 0 ? S.h[l] : which == 1 ? S.a[l] : which == 2 ? S.t[l] : which == 3 ? S.d[l]
                        : which == 4 ? S.z1[l] : which == 5 ? S.z2[l] : which == 6 ? S.out(l)
                        : which == 7 ? S.q[l] : which == 8 ? S.k[l] : S.v[l];
  if (out) {
    const size_t tot = (size_t)h.lv[l].n_n * width;
    if (tot) {
      hipLaunchKernelGGL(k_widen, dim3(nblk(tot)), dim3(kB), 0, s, tot, src, out);
      GMT_LAUNCH_CHECK();
    }
  }
  return width;
}

double nn_norm2(Hier* h, const float* x, size_t n, hipStream_t s) {
  (void)h;
  const unsigned g = 256;
  double* partial = nullptr;
  GMT_HIP(hipMallocAsync((void**)&partial, g * sizeof(double), s));
  hipLaunchKernelGGL(k_norm2, dim3(g), dim3(kB), 0, s, x, n, partial);
  GMT_LAUNCH_CHECK();
  double hp[256];
  GMT_HIP(hipMemcpyAsync(hp, partial, g * sizeof(double), hipMemcpyDeviceToHost, s));
  GMT_HIP(hipFreeAsync(partial, s));
  GMT_HIP(hipStreamSynchronize(s));
  double sum = 0.0;
  for (unsigned k = 0; k < g; ++k) sum += hp[k];
  return sum;
}

// ---------------------------------------------------------------- norm without allocation
// gmt_nn_norm2_noalloc keeps its per-block partial sums in this file-scope
// device array instead of a buffer allocated per call.  Every GPU holds its
// own copy at its own address; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device pointer).  Calls that overlap on one GPU
// share it and race.
constexpr int kNoAllocPartials = 8192;      // 64 KiB of FP64 partial sums (+ the total)
constexpr size_t kNoAllocChunk = 2048;      // values per workgroup (8 per thread)
static __device__ __align__(256) double scratch[kNoAllocPartials + 32];

// total of the g partials into partial[kNoAllocPartials] (one workgroup, fixed order)
__global__ __launch_bounds__(kB) void k_sum_partials(double* __restrict__ partial, int g) {
  __shared__ double sh[kB / 64];
  double v = 0.0;
  for (int k = threadIdx.x; k < g; k += kB) v += partial[k];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kB / 64; ++k) t += sh[k];
    partial[kNoAllocPartials] = t;
  }
}

// The array's device address on the current GPU, looked up once per device
// (with that device current) and kept in a fixed table: no allocation at all.
constexpr int kMaxDevices = 64;
static double* scratch_ptr() {
  static std::mutex mu;
  static double* ptrs[kMaxDevices] = {};
  int dev = 0;
  GMT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) fail(GMT_E_INVAL, "device %d beyond the %d this table covers", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(mu);
  if (!ptrs[dev]) {
    double* p = nullptr;
    GMT_HIP(hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
    ptrs[dev] = p;
  }
  return ptrs[dev];
}

size_t nn_norm2_noalloc_max() { return (size_t)kNoAllocPartials * kNoAllocChunk; }

double nn_norm2_noalloc(const float* x, size_t n, hipStream_t s) {
  if (n > nn_norm2_noalloc_max())
    fail(GMT_E_INVAL, "n = %zu exceeds the %zu values the fixed scratch of gmt_nn_norm2_noalloc covers", n,
         nn_norm2_noalloc_max());
  double* partial = scratch_ptr();
  if (n == 0) return 0.0;
  const unsigned g = (unsigned)((n + kNoAllocChunk - 1) / kNoAllocChunk);
  // every one of the g partials is written by its workgroup and the total
  // overwrites its slot: nothing left from an earlier call is read
  hipLaunchKernelGGL(k_norm2, dim3(g), dim3(kB), 0, s, x, n, partial);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kB), 0, s, partial, (int)g);
  GMT_LAUNCH_CHECK();
  double sum = 0.0;
  GMT_HIP(hipMemcpyAsync(&sum, partial + kNoAllocPartials, sizeof(double), hipMemcpyDeviceToHost, s));
  GMT_HIP(hipStreamSynchronize(s));
  return sum;
}

void nn_ema(float* e, const float* x, size_t n, double decay, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_ema, dim3(nblk(n)), dim3(kB), 0, s, e, x, n, (float)decay);
  GMT_LAUNCH_CHECK();
}

void nn_adamw(float* p, const float* g, float* m, float* v, size_t n, double lr, double b1, double b2, double eps,
              double wd, int step, double gscale, hipStream_t s) {
  if (!n) return;
  const float c1 = (float)(1.0 - std::pow(b1, step)), c2 = (float)(1.0 - std::pow(b2, step));
  hipLaunchKernelGGL(k_adamw, dim3(nblk(n)), dim3(kB), 0, s, n, p, g, m, v, (float)lr, (float)b1, (float)b2, (float)eps,
                     (float)wd, c1, c2, (float)gscale);
  GMT_LAUNCH_CHECK();
}

}  // namespace gmt
