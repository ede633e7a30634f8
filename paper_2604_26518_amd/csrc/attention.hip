// gfx950 kernels of the learned initializer's attention block (Sec. 4.2-4.3):
// serialization of a level's active nodes along a Morton order, and windowed
// multi-head softmax attention with Ra-RoPE, forward and backward.
//
// Serialization (homogenization-aware, Sec. 4.2): the nodes of a level are
// ordered by the Morton code of their coordinates under one of three cyclic
// permutations of the axes -- view 0 (x, y, z), view 1 (y, z, x), view 2
// (z, x, y) -- bit b of the first, second and third coordinate sitting at code
// bits 3b, 3b + 1, 3b + 2.  The codes are distinct, so the order is unique.
// It is built without a sort: one flag per code of the 2^bits cube (bits with
// 2^bits >= N), an exclusive scan of the flags gives every active node its
// rank, and the compacted codes decode back to node ids.
//
// Attention (per window of W consecutive tokens of that order and per head of
// 8 channels): o_i = sum_j softmax_j(q~_i . k~_j / sqrt 8) v_j, with q~, k~ the
// queries and keys after Ra-RoPE (Sec. 4.3, eq. rarope_theta): channel pair k
// of a head turns by 2 pi (k div 3 + 1) p_{k mod 3} / N, p the node's integer
// coordinates on the level and N its period; the angle is reduced in
// integers, (k div 3 + 1) p mod N, so the encoding is exactly periodic.
//
// Every tensor of the block is kept in serialization order ("token" i is the
// node order[i]), so a window is a contiguous run of rows.  One workgroup
// handles one (window, head) pair; a thread owns kPer queries (forward, dq) or
// keys (dk, dv) and streams the other side of the window through LDS in chunks
// of kChunk tokens, so each LDS read serves kPer score evaluations.  The
// softmax is computed online in base 2 in FP32 against a running offset m that
// is raised (and the sums rescaled) only when a score exceeds it by more than 8:
// every term 2^(s - m) stays below 2^8, and the rescaling branch, which a wave
// takes whenever any of its lanes needs it, is rare after the first key.  The
// log-sum-exp m + log2(sum) does not depend on m.  The forward stores it per
// (token, head), and the backward recomputes the probabilities from it.  The
// backward runs as two
// passes, one per query (dq) and one per key (dk, dv), each thread summing its
// own outputs in a fixed order: the gradients are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "common.h"

namespace gmt {

namespace {

constexpr int kHd = 8;        // head dimension
constexpr int kPer = 4;       // queries (or keys) per thread
constexpr int kChunk = 128;   // tokens of the other side staged in LDS at a time
constexpr float kSlack = 8.f; // the running offset may trail the maximum score by 2^8
constexpr int kThreads = 256;
constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ uint16_t tobf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0;  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// the 8 BF16 channels of one head of one token (16 bytes)
__device__ __forceinline__ void load_head(const uint16_t* p, float* x) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[2 * k] = __uint_as_float(w[k] << 16);
    x[2 * k + 1] = __uint_as_float(w[k] & 0xFFFF0000u);
  }
}

__device__ __forceinline__ void load_head(const float* p, float* x) {
  const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
  x[0] = a.x, x[1] = a.y, x[2] = a.z, x[3] = a.w, x[4] = b.x, x[5] = b.y, x[6] = b.z, x[7] = b.w;
}

__device__ __forceinline__ void store_head(float* p, const float* x) {
  reinterpret_cast<float4*>(p)[0] = make_float4(x[0], x[1], x[2], x[3]);
  reinterpret_cast<float4*>(p)[1] = make_float4(x[4], x[5], x[6], x[7]);
}

// cos / sin of the four pair angles of the token at linear index lin = x + N (y + N z)
__device__ __forceinline__ void rope(int lin, int N, float* c, float* s) {
  const int p[3] = {lin % N, (lin / N) % N, lin / (N * N)};
#pragma unroll
  for (int k = 0; k < kHd / 2; ++k) {
    const int r = (int)(((long long)(k / 3 + 1) * p[k % 3]) % N);
    sincospif((float)(2 * r) / (float)N, &s[k], &c[k]);
  }
}

// x <- R(sign theta) x on every channel pair
__device__ __forceinline__ void rotate(float* x, const float* c, const float* s, float sign) {
#pragma unroll
  for (int k = 0; k < kHd / 2; ++k) {
    const float a = x[2 * k], b = x[2 * k + 1], sn = sign * s[k];
    x[2 * k] = c[k] * a - sn * b;
    x[2 * k + 1] = sn * a + c[k] * b;
  }
}

// 2^x on the transcendental unit (v_exp_f32; results below 2^-126 may flush to zero)
__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ float dot8(const float* a, const float4 b0, const float4 b1) {
  float d = a[0] * b0.x;
  d = fmaf(a[1], b0.y, d);
  d = fmaf(a[2], b0.z, d);
  d = fmaf(a[3], b0.w, d);
  d = fmaf(a[4], b1.x, d);
  d = fmaf(a[5], b1.y, d);
  d = fmaf(a[6], b1.z, d);
  return fmaf(a[7], b1.w, d);
}

__device__ __forceinline__ void axpy8(float* y, float a, const float4 x0, const float4 x1) {
  y[0] = fmaf(a, x0.x, y[0]);
  y[1] = fmaf(a, x0.y, y[1]);
  y[2] = fmaf(a, x0.z, y[2]);
  y[3] = fmaf(a, x0.w, y[3]);
  y[4] = fmaf(a, x1.x, y[4]);
  y[5] = fmaf(a, x1.y, y[5]);
  y[6] = fmaf(a, x1.z, y[6]);
  y[7] = fmaf(a, x1.w, y[7]);
}

// ---------------------------------------------------------------- serialization

__device__ __forceinline__ void morton_decode(uint32_t m, int view, int bits, int& x, int& y, int& z) {
  int c[3] = {0, 0, 0};
  for (int b = 0; b < bits; ++b)
#pragma unroll
    for (int s = 0; s < 3; ++s) c[s] |= (int)((m >> (3 * b + s)) & 1u) << b;
  // slot s holds axis (s + view) mod 3
  const int a0 = c[(3 - view) % 3], a1 = c[(4 - view) % 3], a2 = c[(5 - view) % 3];
  x = a0, y = a1, z = a2;
}

__global__ void k_morton_flags(size_t ncode, int view, int bits, int N, const int* __restrict__ node_map,
                               int* __restrict__ flags) {
  const size_t m = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (m >= ncode) return;
  int x, y, z;
  morton_decode((uint32_t)m, view, bits, x, y, z);
  int f = 0;
  if (x < N && y < N && z < N) f = node_map[(size_t)x + (size_t)N * (y + (size_t)N * z)] >= 0;
  flags[m] = f;
}

__global__ void k_morton_order(int n, const int* __restrict__ codes, int view, int bits, int N,
                               const int* __restrict__ node_map, int* __restrict__ order, int* __restrict__ inv,
                               int* __restrict__ ser_lin) {
  const int r = blockIdx.x * kThreads + threadIdx.x;
  if (r >= n) return;
  int x, y, z;
  morton_decode((uint32_t)codes[r], view, bits, x, y, z);
  const int lin = x + N * (y + N * z);
  const int id = node_map[lin];
  order[r] = id;
  inv[id] = r;
  ser_lin[r] = lin;
}

// ---------------------------------------------------------------- forward

// grid (windows, heads), block ceil(W / kPer) threads.  q, k, v, o16: [n][C] BF16,
// o32 [n][C] FP32, lse [n][C / 8] (base 2, of the scores scaled by log2(e) / sqrt 8).
__global__ __launch_bounds__(kThreads) void k_attn_fwd(int n, int W, int C, int N, const int* __restrict__ ser_lin,
                                                       const uint16_t* __restrict__ q, const uint16_t* __restrict__ k,
                                                       const uint16_t* __restrict__ v, float* __restrict__ o32,
                                                       uint16_t* __restrict__ o16, float* __restrict__ lse) {
  __shared__ float4 kv[kChunk][4];  // k~ (2 float4), v (2 float4)
  const int h = blockIdx.y, heads = C / kHd;
  const int w0 = blockIdx.x * W, wn = min(W, n - w0);
  const int nt = blockDim.x;
  const float scale = kLog2e * 0.35355339059327373f;  // log2(e) / sqrt(8)
  float qs[kPer][kHd], acc[kPer][kHd], mx[kPer], l[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int j = threadIdx.x + r * nt;
    float c[4], s[4];
    if (j < wn) {
      load_head(q + (size_t)(w0 + j) * C + kHd * h, qs[r]);
      rope(ser_lin[w0 + j], N, c, s);
      rotate(qs[r], c, s, 1.f);
    } else {
#pragma unroll
      for (int d = 0; d < kHd; ++d) qs[r][d] = 0.f;
    }
#pragma unroll
    for (int d = 0; d < kHd; ++d) {
      qs[r][d] *= scale;
      acc[r][d] = 0.f;
    }
    mx[r] = -INFINITY;
    l[r] = 0.f;
  }
  for (int c0 = 0; c0 < wn; c0 += kChunk) {
    const int cn = min(kChunk, wn - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cn; j += nt) {
      const int i = w0 + c0 + j;
      float kk[kHd], vv[kHd], c[4], s[4];
      load_head(k + (size_t)i * C + kHd * h, kk);
      load_head(v + (size_t)i * C + kHd * h, vv);
      rope(ser_lin[i], N, c, s);
      rotate(kk, c, s, 1.f);
      kv[j][0] = make_float4(kk[0], kk[1], kk[2], kk[3]);
      kv[j][1] = make_float4(kk[4], kk[5], kk[6], kk[7]);
      kv[j][2] = make_float4(vv[0], vv[1], vv[2], vv[3]);
      kv[j][3] = make_float4(vv[4], vv[5], vv[6], vv[7]);
    }
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < cn; ++j) {
      const float4 k0 = kv[j][0], k1 = kv[j][1], v0 = kv[j][2], v1 = kv[j][3];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const float sc = dot8(qs[r], k0, k1);
        if (sc > mx[r] + kSlack) {
          const float f = ex2(mx[r] - sc);
          l[r] *= f;
#pragma unroll
          for (int d = 0; d < kHd; ++d) acc[r][d] *= f;
          mx[r] = sc;
        }
        const float p = ex2(sc - mx[r]);
        l[r] += p;
        axpy8(acc[r], p, v0, v1);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int j = threadIdx.x + r * nt;
    if (j >= wn) continue;
    const size_t i = (size_t)(w0 + j);
    const float inv = 1.f / l[r];
    float o[kHd];
#pragma unroll
    for (int d = 0; d < kHd; ++d) o[d] = acc[r][d] * inv;
    store_head(o32 + i * C + kHd * h, o);
    uint4 pk;
    pk.x = (uint32_t)tobf(o[0]) | ((uint32_t)tobf(o[1]) << 16);
    pk.y = (uint32_t)tobf(o[2]) | ((uint32_t)tobf(o[3]) << 16);
    pk.z = (uint32_t)tobf(o[4]) | ((uint32_t)tobf(o[5]) << 16);
    pk.w = (uint32_t)tobf(o[6]) | ((uint32_t)tobf(o[7]) << 16);
    *reinterpret_cast<uint4*>(o16 + i * C + kHd * h) = pk;
    lse[i * heads + h] = mx[r] + log2f(l[r]);
  }
}

// ---------------------------------------------------------------- backward
// With P the window's probabilities, dO = go and D_i = go_i . o_i:
//   dS_ij = P_ij (go_i . v_j - D_i) / sqrt 8,  dq~_i = sum_j dS_ij k~_j,
//   dk~_j = sum_i dS_ij q~_i,  dv_j = sum_i P_ij go_i,
// and dq, dk are dq~, dk~ turned back by -theta (the rotation is orthogonal).

// pass A: one thread per kPer queries; keys and values of the window through LDS
__global__ __launch_bounds__(kThreads) void k_attn_bwd_q(int n, int W, int C, int N, const int* __restrict__ ser_lin,
                                                         const uint16_t* __restrict__ q,
                                                         const uint16_t* __restrict__ k,
                                                         const uint16_t* __restrict__ v,
                                                         const float* __restrict__ o32,
                                                         const float* __restrict__ lse,
                                                         const float* __restrict__ go, float* __restrict__ dq) {
  __shared__ float4 kv[kChunk][4];
  const int h = blockIdx.y, heads = C / kHd;
  const int w0 = blockIdx.x * W, wn = min(W, n - w0);
  const int nt = blockDim.x;
  const float scale = kLog2e * 0.35355339059327373f;
  float qs[kPer][kHd], g[kPer][kHd], acc[kPer][kHd], Dq[kPer], lq[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int j = threadIdx.x + r * nt;
#pragma unroll
    for (int d = 0; d < kHd; ++d) acc[r][d] = 0.f;
    if (j < wn) {
      const size_t i = (size_t)(w0 + j);
      float c[4], s[4], o[kHd];
      load_head(q + i * C + kHd * h, qs[r]);
      rope(ser_lin[i], N, c, s);
      rotate(qs[r], c, s, 1.f);
      load_head(go + i * C + kHd * h, g[r]);
      load_head(o32 + i * C + kHd * h, o);
      float D = 0.f;
#pragma unroll
      for (int d = 0; d < kHd; ++d) D = fmaf(g[r][d], o[d], D);
      Dq[r] = D;
      lq[r] = lse[i * heads + h];
    } else {
#pragma unroll
      for (int d = 0; d < kHd; ++d) qs[r][d] = g[r][d] = 0.f;
      Dq[r] = 0.f;
      lq[r] = 0.f;
    }
#pragma unroll
    for (int d = 0; d < kHd; ++d) qs[r][d] *= scale;
  }
  for (int c0 = 0; c0 < wn; c0 += kChunk) {
    const int cn = min(kChunk, wn - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cn; j += nt) {
      const int i = w0 + c0 + j;
      float kk[kHd], vv[kHd], c[4], s[4];
      load_head(k + (size_t)i * C + kHd * h, kk);
      load_head(v + (size_t)i * C + kHd * h, vv);
      rope(ser_lin[i], N, c, s);
      rotate(kk, c, s, 1.f);
      kv[j][0] = make_float4(kk[0], kk[1], kk[2], kk[3]);
      kv[j][1] = make_float4(kk[4], kk[5], kk[6], kk[7]);
      kv[j][2] = make_float4(vv[0], vv[1], vv[2], vv[3]);
      kv[j][3] = make_float4(vv[4], vv[5], vv[6], vv[7]);
    }
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < cn; ++j) {
      const float4 k0 = kv[j][0], k1 = kv[j][1], v0 = kv[j][2], v1 = kv[j][3];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const float p = ex2(dot8(qs[r], k0, k1) - lq[r]);
        const float ds = p * (dot8(g[r], v0, v1) - Dq[r]);
        axpy8(acc[r], ds, k0, k1);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int j = threadIdx.x + r * nt;
    if (j >= wn) continue;
    const size_t i = (size_t)(w0 + j);
    float c[4], s[4];
    rope(ser_lin[i], N, c, s);
#pragma unroll
    for (int d = 0; d < kHd; ++d) acc[r][d] *= 0.35355339059327373f;
    rotate(acc[r], c, s, -1.f);
    store_head(dq + i * C + kHd * h, acc[r]);
  }
}

// pass B: one thread per kPer keys; per query q~ (scaled), go, lse and D through LDS
__global__ __launch_bounds__(kThreads) void k_attn_bwd_kv(int n, int W, int C, int N,
                                                          const int* __restrict__ ser_lin,
                                                          const uint16_t* __restrict__ q,
                                                          const uint16_t* __restrict__ k,
                                                          const uint16_t* __restrict__ v,
                                                          const float* __restrict__ o32,
                                                          const float* __restrict__ lse,
                                                          const float* __restrict__ go, float* __restrict__ dk,
                                                          float* __restrict__ dv) {
  __shared__ float4 qg[kChunk][4];  // q~ scaled (2 float4), go (2 float4)
  __shared__ float2 ld[kChunk];     // lse, D
  const int h = blockIdx.y, heads = C / kHd;
  const int w0 = blockIdx.x * W, wn = min(W, n - w0);
  const int nt = blockDim.x;
  const float scale = kLog2e * 0.35355339059327373f;
  float kk[kPer][kHd], vv[kPer][kHd], ak[kPer][kHd], av[kPer][kHd];
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int j = threadIdx.x + r * nt;
#pragma unroll
    for (int d = 0; d < kHd; ++d) ak[r][d] = av[r][d] = 0.f;
    if (j < wn) {
      const size_t i = (size_t)(w0 + j);
      float c[4], s[4];
      load_head(k + i * C + kHd * h, kk[r]);
      load_head(v + i * C + kHd * h, vv[r]);
      rope(ser_lin[i], N, c, s);
      rotate(kk[r], c, s, 1.f);
    } else {
#pragma unroll
      for (int d = 0; d < kHd; ++d) kk[r][d] = vv[r][d] = 0.f;
    }
  }
  for (int c0 = 0; c0 < wn; c0 += kChunk) {
    const int cn = min(kChunk, wn - c0);
    __syncthreads();
    for (int j = threadIdx.x; j < cn; j += nt) {
      const size_t i = (size_t)(w0 + c0 + j);
      float qq[kHd], gg[kHd], o[kHd], c[4], s[4];
      load_head(q + i * C + kHd * h, qq);
      rope(ser_lin[i], N, c, s);
      rotate(qq, c, s, 1.f);
      load_head(go + i * C + kHd * h, gg);
      load_head(o32 + i * C + kHd * h, o);
      float D = 0.f;
#pragma unroll
      for (int d = 0; d < kHd; ++d) D = fmaf(gg[d], o[d], D);
      qg[j][0] = make_float4(qq[0] * scale, qq[1] * scale, qq[2] * scale, qq[3] * scale);
      qg[j][1] = make_float4(qq[4] * scale, qq[5] * scale, qq[6] * scale, qq[7] * scale);
      qg[j][2] = make_float4(gg[0], gg[1], gg[2], gg[3]);
      qg[j][3] = make_float4(gg[4], gg[5], gg[6], gg[7]);
      ld[j] = make_float2(lse[i * heads + h], D);
    }
    __syncthreads();
#pragma unroll 2
    for (int j = 0; j < cn; ++j) {
      const float4 q0 = qg[j][0], q1 = qg[j][1], g0 = qg[j][2], g1 = qg[j][3];
      const float2 lD = ld[j];
#pragma unroll
      for (int r = 0; r < kPer; ++r) {
        const float p = ex2(dot8(kk[r], q0, q1) - lD.x);
        axpy8(av[r], p, g0, g1);
        const float ds = p * (dot8(vv[r], g0, g1) - lD.y);
        axpy8(ak[r], ds, q0, q1);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int j = threadIdx.x + r * nt;
    if (j >= wn) continue;
    const size_t i = (size_t)(w0 + j);
    float c[4], s[4];
    rope(ser_lin[i], N, c, s);
    // ak sums ds * (q~ log2(e) / sqrt 8); dk~ = sum ds q~ / sqrt 8 = ak / log2(e)
#pragma unroll
    for (int d = 0; d < kHd; ++d) ak[r][d] *= 0.69314718055994531f;
    rotate(ak[r], c, s, -1.f);
    store_head(dk + i * C + kHd * h, ak[r]);
    store_head(dv + i * C + kHd * h, av[r]);
  }
}

inline unsigned blocks(size_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

void check_shape(int n, int W, int C) {
  if (n < 0 || C % kHd || C <= 0 || W <= 0 || W > kPer * kThreads)
    fail(GMT_E_INVAL, "attention of %d tokens, %d channels, window %d is outside the kernel's shapes", n, C, W);
}

}  // namespace

int attention_window(int level) { return std::min(256 << std::min(level, 2), 1024); }

void attention_serialize(const int* node_map, int N, int n, int view, int* order, int* inv, int* ser_lin,
                         hipStream_t s) {
  if (n <= 0) return;
  if (view < 0 || view > 2) fail(GMT_E_INVAL, "serialization view %d outside 0..2", view);
  int bits = 0;
  while ((1 << bits) < N) ++bits;
  if (bits > 10) fail(GMT_E_INVAL, "serialization supports levels up to 1024^3 (N = %d)", N);
  const size_t ncode = (size_t)1 << (3 * bits);
  int *flags = nullptr, *map = nullptr, *codes = nullptr, *scr = nullptr, *total = nullptr;
  GMT_HIP(hipMalloc((void**)&flags, ncode * sizeof(int)));
  GMT_HIP(hipMalloc((void**)&map, ncode * sizeof(int)));
  GMT_HIP(hipMalloc((void**)&codes, (size_t)n * sizeof(int)));
  GMT_HIP(hipMalloc((void**)&scr, scan_scratch_ints(ncode) * sizeof(int)));
  GMT_HIP(hipMalloc((void**)&total, sizeof(int)));
  hipLaunchKernelGGL(k_morton_flags, dim3(blocks(ncode)), dim3(kThreads), 0, s, ncode, view, bits, N, node_map,
                     flags);
  GMT_LAUNCH_CHECK();
  const int64_t cnt = scan_compact(flags, ncode, map, codes, scr, total, s);
  if (cnt != n) fail(GMT_E_STATE, "serialization found %lld of %d nodes", (long long)cnt, n);
  hipLaunchKernelGGL(k_morton_order, dim3(blocks(n)), dim3(kThreads), 0, s, n, codes, view, bits, N, node_map, order,
                     inv, ser_lin);
  GMT_LAUNCH_CHECK();
  GMT_HIP(hipStreamSynchronize(s));
  GMT_HIP(hipFree(flags));
  GMT_HIP(hipFree(map));
  GMT_HIP(hipFree(codes));
  GMT_HIP(hipFree(scr));
  GMT_HIP(hipFree(total));
}

void attention_forward(int n, int W, int C, int N, const int* ser_lin, const uint16_t* q, const uint16_t* k,
                       const uint16_t* v, float* o32, uint16_t* o16, float* lse, hipStream_t s) {
  check_shape(n, W, C);
  if (n == 0) return;
  const dim3 grid((unsigned)((n + W - 1) / W), (unsigned)(C / kHd));
  const dim3 block((unsigned)((W + kPer - 1) / kPer));
  hipLaunchKernelGGL(k_attn_fwd, grid, block, 0, s, n, W, C, N, ser_lin, q, k, v, o32, o16, lse);
  GMT_LAUNCH_CHECK();
}

void attention_backward(int n, int W, int C, int N, const int* ser_lin, const uint16_t* q, const uint16_t* k,
                        const uint16_t* v, const float* o32, const float* lse, const float* go, float* dq, float* dk,
                        float* dv, hipStream_t s) {
  check_shape(n, W, C);
  if (n == 0) return;
  const dim3 grid((unsigned)((n + W - 1) / W), (unsigned)(C / kHd));
  const dim3 block((unsigned)((W + kPer - 1) / kPer));
  hipLaunchKernelGGL(k_attn_bwd_q, grid, block, 0, s, n, W, C, N, ser_lin, q, k, v, o32, lse, go, dq);
  GMT_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_attn_bwd_kv, grid, block, 0, s, n, W, C, N, ser_lin, q, k, v, o32, lse, go, dk, dv);
  GMT_LAUNCH_CHECK();
}

}  // namespace gmt
