// Learned screener kernels: hashed subtree features, a bf16 MLP whose products
// run on MFMA (v_mfma_f32_32x32x16_bf16, fp32 accumulation), its backward pass,
// BCE-with-logits on the two coverage fractions, AdamW, and top-k selection.
//
// The screener ranks refinement candidates so that only the best fraction is
// evaluated exactly; the exact engine stays the judge of every count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "kb_handle.h"

namespace hth {

// ---------------------------------------------------------------------------
// features: Merkle FNV-1a over the postfix nodes of each hypothesis
// ---------------------------------------------------------------------------
constexpr uint64_t kFnvOffset = 0xCBF29CE484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001B3ull;
constexpr uint32_t kFeatDim = 4096;

__device__ __forceinline__ uint64_t fnv_bytes(uint64_t h, uint64_t v, int n) {
  for (int i = 0; i < n; ++i) {
    h ^= (v >> (8 * i)) & 0xFFu;
    h *= kFnvPrime;
  }
  return h;
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {   // splitmix64 finaliser
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// header bytes of a node: op, inv, arity (2 LE), arg (4 LE), q (4 LE), with the
// fields a construct does not use set to zero
__device__ __forceinline__ uint64_t node_header_hash(const hth_node& n) {
  const uint32_t op = n.op;
  const bool value_op = op >= HTH_DATA_EQ && op <= HTH_NUM_EQ;   // EXACT and numeric concrete roles
  const bool uses_arg = op == HTH_ATOM || (op >= HTH_EXISTS && op <= HTH_DATA_LE) || value_op;
  const bool uses_q = (op >= HTH_ATLEAST && op <= HTH_EXACTLY) || op == HTH_DATA_GE || op == HTH_DATA_LE ||
                      value_op;
  const bool uses_inv = op >= HTH_EXISTS && op <= HTH_EXACTLY;
  const uint32_t arity = (op == HTH_AND || op == HTH_OR) ? n.arity : 0;
  uint32_t q;
  memcpy(&q, &n.q, 4);
  uint64_t h = kFnvOffset;
  h = fnv_bytes(h, op, 1);
  h = fnv_bytes(h, uses_inv ? n.inv : 0, 1);
  h = fnv_bytes(h, arity, 2);
  h = fnv_bytes(h, uses_arg ? n.arg : 0, 4);
  h = fnv_bytes(h, uses_q ? q : 0, 4);
  return h;
}

// one thread per hypothesis; hash[i] holds node i's subtree hash, feat[i] its
// feature index (hash mod 4096).  Malformed child indices set *bad and hash 0.
__global__ void k_features(const hth_node* __restrict__ nodes, const uint32_t* __restrict__ offs,
                           const uint32_t* __restrict__ children, uint32_t n_children,
                           uint32_t n_hyps, uint64_t* __restrict__ hash, uint16_t* __restrict__ feat,
                           uint32_t* __restrict__ bad) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= n_hyps) return;
  const uint32_t b = offs[h], e = offs[h + 1];
  for (uint32_t i = b; i < e; ++i) {
    const hth_node n = nodes[i];
    const uint32_t li = i - b;
    uint64_t v = node_header_hash(n);
    // the DL constructs; set-table leaves carry no syntax
    bool ok = n.op <= HTH_DATA_LE || (n.op >= HTH_DATA_EQ && n.op <= HTH_NUM_EQ);
    if (n.op == HTH_NOT || (n.op >= HTH_EXISTS && n.op <= HTH_EXACTLY)) {
      ok = ok && n.child < li;
      v = fnv_bytes(v, ok ? hash[b + n.child] : 0ull, 8);
    } else if (n.op == HTH_AND || n.op == HTH_OR) {
      uint64_t s = 0;
      ok = ok && (uint64_t)n.child + n.arity <= n_children;
      for (uint32_t j = 0; ok && j < n.arity; ++j) {
        const uint32_t c = children[n.child + j];
        ok = c < li;
        if (ok) s += mix64(hash[b + c]);
      }
      v = fnv_bytes(v, s, 8);
    }
    if (!ok) {
      atomicOr(bad, 1u);
      v = 0;
    }
    hash[i] = v;
    feat[i] = (uint16_t)(v & (kFeatDim - 1));
  }
}

// dense bf16 feature rows: x[r][f] = number of subtrees of hypothesis row0 + r
// whose feature index is f (small integers, exact in bf16)
__global__ void __launch_bounds__(256)
k_densify(const uint16_t* __restrict__ feat, const uint32_t* __restrict__ offs, uint32_t row0,
          uint32_t n_rows, const uint16_t* __restrict__ pfeat, const uint32_t* __restrict__ poffs,
          const uint32_t* __restrict__ pidx, uint32_t context, __bf16* __restrict__ x) {
  __shared__ int32_t cnt[kFeatDim];
  const uint32_t r = blockIdx.x;
  if (r >= n_rows) return;
  for (uint32_t i = threadIdx.x; i < kFeatDim; i += 256) cnt[i] = 0;
  __syncthreads();
  const uint32_t b = offs[row0 + r], e = offs[row0 + r + 1];
  for (uint32_t i = b + threadIdx.x; i < e; i += 256) atomicAdd(&cnt[feat[i] & (kFeatDim - 1)], 1);
  if (pidx) {   // minus the parent's subtrees: what the refinement added or changed
    const uint32_t p = pidx[row0 + r];
    const uint32_t pb = poffs[p], pe = poffs[p + 1];
    for (uint32_t i = pb + threadIdx.x; i < pe; i += 256) atomicSub(&cnt[pfeat[i] & (kFeatDim - 1)], 1);
    // the parent itself, in the other half of the index space (top bit flipped)
    if (context)
      for (uint32_t i = pb + threadIdx.x; i < pe; i += 256)
        atomicAdd(&cnt[(pfeat[i] & (kFeatDim - 1)) ^ (kFeatDim / 2)], 1);
  }
  __syncthreads();
  __bf16* row = x + (size_t)r * kFeatDim;
  for (uint32_t i = threadIdx.x; i < kFeatDim; i += 256) row[i] = (__bf16)(float)cnt[i];
}

// ---------------------------------------------------------------------------
// bf16 GEMM on MFMA: C[M][N] = sum_k A[m][k] B[k][n], fp32 accumulation
//   TA = 0: A stored [M][K] (lda >= K);  TA = 1: A stored [K][M] (A^T given)
//   TB = 0: B stored [K][N] (ldb >= N);  TB = 1: B stored [N][K]
// Epilogue: + bias[n]; ReLU; * (mask[m][n] > 0); outputs fp32 and/or bf16.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 128, BN = 128, BK = 32, LDK = BK + 8;   // LDS rows padded by 16 bytes

struct GemmEpi {
  const float* bias;     // [N] or null
  int relu;              // 1: max(x, 0)
  const __bf16* mask;    // [M][ldm] or null: zero where mask <= 0
  int ldm;
  float* c32;            // [M][ldc] or null
  int ldc;
  __bf16* cbf;           // [M][ldcb] or null
  int ldcb;
};

template <int TA, int TB>
__global__ void __launch_bounds__(256)
k_gemm_bf16(int M, int N, int K, const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B,
            int ldb, GemmEpi ep) {
  __shared__ __bf16 As[BM][LDK];
  __shared__ __bf16 Bs[BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;            // 2 x 2 waves, 64 x 64 each
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  for (int k0 = 0; k0 < K; k0 += BK) {
    // ---- stage A tile as As[m][k]
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int chunk = tid + 256 * c;            // 512 chunks of 8 elements
      if (TA == 0) {
        const int m = chunk >> 2, kk = (chunk & 3) * 8;
        const int gm = m0 + m, gk = k0 + kk;
        bf16x8 v;
        if (gm < M && gk < K) v = *reinterpret_cast<const bf16x8*>(A + (size_t)gm * lda + gk);
        else
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.f;
        *reinterpret_cast<bf16x8*>(&As[m][kk]) = v;
      } else {
        const int kk = chunk >> 4, m = (chunk & 15) * 8;
        const int gm = m0 + m, gk = k0 + kk;
        bf16x8 v;
        if (gm < M && gk < K) v = *reinterpret_cast<const bf16x8*>(A + (size_t)gk * lda + gm);
        else
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) As[m + i][kk] = v[i];
      }
    }
    // ---- stage B tile as Bs[n][k]
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int chunk = tid + 256 * c;
      if (TB == 1) {
        const int n = chunk >> 2, kk = (chunk & 3) * 8;
        const int gn = n0 + n, gk = k0 + kk;
        bf16x8 v;
        if (gn < N && gk < K) v = *reinterpret_cast<const bf16x8*>(B + (size_t)gn * ldb + gk);
        else
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.f;
        *reinterpret_cast<bf16x8*>(&Bs[n][kk]) = v;
      } else {
        const int kk = chunk >> 4, n = (chunk & 15) * 8;
        const int gn = n0 + n, gk = k0 + kk;
        bf16x8 v;
        if (gn < N && gk < K) v = *reinterpret_cast<const bf16x8*>(B + (size_t)gk * ldb + gn);
        else
#pragma unroll
          for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.f;
#pragma unroll
        for (int i = 0; i < 8; ++i) Bs[n + i][kk] = v[i];
      }
    }
    __syncthreads();
    // ---- 2 x 2 tiles of 32 x 32, two k-steps of 16
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 64 + i * 32 + (lane & 31)][ks + 8 * (lane >> 5)]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 64 + j * 32 + (lane & 31)][ks + 8 * (lane >> 5)]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // ---- epilogue: register r of lane l holds row 8(r/4) + 4(l/32) + r%4, column l%32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int gm = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int gn = n0 + wn * 64 + j * 32 + (lane & 31);
        if (gm >= M || gn >= N) continue;
        float v = acc[i][j][r];
        if (ep.bias) v += ep.bias[gn];
        if (ep.relu) v = fmaxf(v, 0.f);
        if (ep.mask && !((float)ep.mask[(size_t)gm * ep.ldm + gn] > 0.f)) v = 0.f;
        if (ep.c32) ep.c32[(size_t)gm * ep.ldc + gn] = v;
        if (ep.cbf) ep.cbf[(size_t)gm * ep.ldcb + gn] = (__bf16)v;
      }
}

// ---------------------------------------------------------------------------
// The same product for A [M][K] and B given as [N][K] (both operands
// contiguous along K), the forward layers' layout: every tile is staged with
// 16-byte loads and stores.  Tiles of 128 x 128 x 64; while the MFMAs work
// on the k-tile in LDS, the next k-tile's global loads are already in flight
// into registers.  4 waves, each a 64 x 64 quarter of the tile as 2 x 2
// products of 32 x 32 on v_mfma_f32_32x32x16_bf16.
// ---------------------------------------------------------------------------
constexpr int NBK = 64, NLDK = NBK + 8;   // LDS rows padded by 16 bytes
__global__ void __launch_bounds__(256)
k_gemm_nt(int M, int N, int K, const __bf16* __restrict__ A, int lda, const __bf16* __restrict__ B, int ldb,
          GemmEpi ep) {
  __shared__ __bf16 As[BM][NLDK];
  __shared__ __bf16 Bs[BN][NLDK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;
  // a tile row holds 64 k = 8 chunks of 8; thread t stages chunks t + 256 c
  bf16x8 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int chunk = tid + 256 * c, row = chunk >> 3, kk = (chunk & 7) * 8;
      const int gk = k0 + kk;
      const int gm = m0 + row, gn = n0 + row;
      if (gm < M && gk < K) ra[c] = *reinterpret_cast<const bf16x8*>(A + (size_t)gm * lda + gk);
      else
#pragma unroll
        for (int i = 0; i < 8; ++i) ra[c][i] = (__bf16)0.f;
      if (gn < N && gk < K) rb[c] = *reinterpret_cast<const bf16x8*>(B + (size_t)gn * ldb + gk);
      else
#pragma unroll
        for (int i = 0; i < 8; ++i) rb[c][i] = (__bf16)0.f;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int chunk = tid + 256 * c, row = chunk >> 3, kk = (chunk & 7) * 8;
      *reinterpret_cast<bf16x8*>(&As[row][kk]) = ra[c];
      *reinterpret_cast<bf16x8*>(&Bs[row][kk]) = rb[c];
    }
  };
  load(0);
  stage();
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += NBK) {
    const bool more = k0 + NBK < K;
    if (more) load(k0 + NBK);                     // in flight during the MFMAs below
#pragma unroll
    for (int ks = 0; ks < NBK; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&As[wm * 64 + i * 32 + (lane & 31)][ks + 8 * (lane >> 5)]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 64 + j * 32 + (lane & 31)][ks + 8 * (lane >> 5)]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      stage();
      __syncthreads();
    }
  }
  // epilogue: register r of lane l holds row 8(r/4) + 4(l/32) + r%4, column l%32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int gm = m0 + wm * 64 + i * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int gn = n0 + wn * 64 + j * 32 + (lane & 31);
        if (gm >= M || gn >= N) continue;
        float v = acc[i][j][r];
        if (ep.bias) v += ep.bias[gn];
        if (ep.relu) v = fmaxf(v, 0.f);
        if (ep.mask && !((float)ep.mask[(size_t)gm * ep.ldm + gn] > 0.f)) v = 0.f;
        if (ep.c32) ep.c32[(size_t)gm * ep.ldc + gn] = v;
        if (ep.cbf) ep.cbf[(size_t)gm * ep.ldcb + gn] = (__bf16)v;
      }
}

// dst[c][r] = src[r][c] for a rows x cols bf16 matrix (32 x 32 tiles through LDS)
__global__ void __launch_bounds__(256)
k_transpose_bf16(const __bf16* __restrict__ src, int rows, int cols, __bf16* __restrict__ dst) {
  __shared__ __bf16 t[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int i = ty; i < 32; i += 8)
    if (r0 + i < rows && c0 + tx < cols) t[i][tx] = src[(size_t)(r0 + i) * cols + c0 + tx];
  __syncthreads();
  for (int i = ty; i < 32; i += 8)
    if (c0 + i < cols && r0 + tx < rows) dst[(size_t)(c0 + i) * rows + r0 + tx] = t[tx][i];
}

// ---------------------------------------------------------------------------
// the 2-wide output layer, loss and its gradient
// ---------------------------------------------------------------------------
// z[b][o] = sum_k h[b][k] w[k][o] + bias[o]; with targets y: per element
// either BCE-with-logits, dz = (sigmoid(z) - y) * scale (kind 0), or the
// squared error (z - y)^2 / 2, dz = (z - y) * scale (kind 1); loss summed
// into *loss.
__global__ void k_head_forward(const __bf16* __restrict__ h, int Bn, int Kd, const float* __restrict__ w,
                               const float* __restrict__ bias, float* __restrict__ z,
                               const float* __restrict__ y, float* __restrict__ dz, float scale,
                               float* __restrict__ loss, int kind) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (b < Bn) {
    float z0 = bias[0], z1 = bias[1];
    const __bf16* hr = h + (size_t)b * Kd;
    for (int k = 0; k < Kd; ++k) {
      const float hv = (float)hr[k];
      z0 = fmaf(hv, w[2 * k], z0);
      z1 = fmaf(hv, w[2 * k + 1], z1);
    }
    z[2 * b] = z0;
    z[2 * b + 1] = z1;
    if (y) {
      const float zz[2] = {z0, z1};
      for (int o = 0; o < 2; ++o) {
        const float t = y[2 * b + o], v = zz[o];
        if (kind == 0) {
          l += fmaxf(v, 0.f) - v * t + log1pf(expf(-fabsf(v)));
          dz[2 * b + o] = (1.f / (1.f + expf(-v)) - t) * scale;
        } else {
          l += 0.5f * (v - t) * (v - t);
          dz[2 * b + o] = (v - t) * scale;
        }
      }
    }
  }
  if (y && loss) {
    for (int d = 32; d >= 1; d >>= 1) l += __shfl_xor(l, d, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, l);
  }
}

// predicted F1 of each candidate from its two outputs, F1 = 2p / (p + q + |P|),
// with (P_b, N_b) the candidate's base coverage (its parent's) or (|P|, |Ng|):
//   kind 0: the outputs are logits of the kept shares, p = sigmoid(z0) P_b,
//           q = sigmoid(z1) N_b;
//   kind 1: the outputs are log(1 + removed count), p = P_b - expm1(z0) and
//           q = N_b - expm1(z1), each clamped to [0, base].
__global__ void k_head_score(const float* __restrict__ z, int Bn, float n_pos, float n_neg,
                             const uint32_t* __restrict__ base, int kind, float* __restrict__ score) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bn) return;
  const float bp = base ? (float)base[2 * b] : n_pos, bn = base ? (float)base[2 * b + 1] : n_neg;
  float p, q;
  if (kind == 0) {
    p = bp / (1.f + expf(-z[2 * b]));
    q = bn / (1.f + expf(-z[2 * b + 1]));
  } else {
    p = fminf(fmaxf(bp - expm1f(fmaxf(z[2 * b], 0.f)), 0.f), bp);
    q = fminf(fmaxf(bn - expm1f(fmaxf(z[2 * b + 1], 0.f)), 0.f), bn);
  }
  const float den = p + q + n_pos;
  score[b] = den > 0.f ? 2.f * p / den : 0.f;
}

// dw[k][o] = sum_b h[b][k] dz[b][o] (one block per k); dh[b][k] = (dz[b] . w[k]) * (h[b][k] > 0)
__global__ void __launch_bounds__(256)
k_head_backward(const __bf16* __restrict__ h, int Bn, int Kd, const float* __restrict__ w,
                const float* __restrict__ dz, float* __restrict__ dw, __bf16* __restrict__ dh) {
  const int k = blockIdx.x;
  float s0 = 0.f, s1 = 0.f;
  const float w0 = w[2 * k], w1 = w[2 * k + 1];
  for (int b = threadIdx.x; b < Bn; b += 256) {
    const float hv = (float)h[(size_t)b * Kd + k];
    const float d0 = dz[2 * b], d1 = dz[2 * b + 1];
    s0 = fmaf(hv, d0, s0);
    s1 = fmaf(hv, d1, s1);
    dh[(size_t)b * Kd + k] = (__bf16)(hv > 0.f ? fmaf(d0, w0, d1 * w1) : 0.f);
  }
  __shared__ float r0[256], r1[256];
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if (threadIdx.x < d) {
      r0[threadIdx.x] += r0[threadIdx.x + d];
      r1[threadIdx.x] += r1[threadIdx.x + d];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dw[2 * k] = r0[0];
    dw[2 * k + 1] = r1[0];
  }
}

// out[n] = sum_m d[m][n] (bias gradients), one thread per column
// Column sums of a row-major M x N matrix: a block per 64 columns, lane c of
// each of its waves on column c (one coalesced row segment per wave and
// step), wave w on rows w, w + 4, ...; the four waves' sums are added in a
// fixed order, so the result does not depend on scheduling.
template <typename T>
__global__ void __launch_bounds__(256) k_colsum(const T* __restrict__ d, int M, int N, float* __restrict__ out) {
  __shared__ float part[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (n < N) {
#pragma unroll 8
    for (int m = wv; m < M; m += 4) s += (float)d[(size_t)m * N + n];
  }
  part[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && n < N) out[n] = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// AdamW on fp32 master weights (decoupled weight decay), with a bf16 copy
__global__ void k_adamw(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, __bf16* __restrict__ pbf, size_t n, float lr, float b1,
                        float b2, float eps, float wd, float c1, float c2) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    float pi = p[i] * (1.f - lr * wd);
    pi -= lr * mh / (sqrtf(vh) + eps);
    p[i] = pi;
    if (pbf) pbf[i] = (__bf16)pi;
  }
}

__global__ void k_to_bf16(const float* __restrict__ s, __bf16* __restrict__ d, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) d[i] = (__bf16)s[i];
}

// ---------------------------------------------------------------------------
// top-k by a float score: radix select on the order-preserving key, then a
// stable compaction (ties at the threshold resolved by index)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fkey(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if (f != f) return 0;                       // NaN ranks last
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// histogram of key bits [shift, shift+16) among keys whose higher bits equal prefix
__global__ void k_topk_hist(const float* __restrict__ s, uint32_t n, uint32_t shift, uint32_t prefix,
                            uint32_t pmask, uint32_t* __restrict__ hist) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t step = gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    const uint32_t k = fkey(s[i]);
    if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 0xFFFFu], 1u);
  }
}

// keys > thr go out; keys == thr go out until `eq_take` of them (in index order
// is not required: the host asks for exactly k and the equal ones are taken by
// a counter, so which equal keys are chosen is the atomics' order)
__global__ void k_topk_collect(const float* __restrict__ s, uint32_t n, uint32_t thr, uint32_t eq_take,
                               uint32_t* __restrict__ out, uint32_t* __restrict__ cnt) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t step = gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    const uint32_t k = fkey(s[i]);
    if (k > thr) {
      out[atomicAdd(&cnt[0], 1u)] = i;
    } else if (k == thr) {
      const uint32_t t = atomicAdd(&cnt[1], 1u);
      if (t < eq_take) out[atomicAdd(&cnt[0], 1u)] = i;
    }
  }
}

}  // namespace hth

using namespace hth;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" hth_status hth_features(const hth_node* d_nodes, const uint32_t* d_hyp_node_offsets,
                                   uint32_t n_hyps, const uint32_t* d_children, uint32_t n_children,
                                   uint64_t* d_hash, uint16_t* d_feat, uint32_t* d_bad, void* stream) {
  if (!d_nodes || !d_hyp_node_offsets || !d_hash || !d_feat || !d_bad)
    return fail(HTH_E_INVALID, "NULL argument");
  if (n_children && !d_children) return fail(HTH_E_INVALID, "children is NULL");
  if (!n_hyps) return HTH_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HTH_HIP(hipMemsetAsync(d_bad, 0, 4, st));
  hipLaunchKernelGGL(k_features, dim3((n_hyps + 255) / 256), dim3(256), 0, st, d_nodes,
                     d_hyp_node_offsets, d_children, n_children, n_hyps, d_hash, d_feat, d_bad);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_densify(const uint16_t* d_feat, const uint32_t* d_hyp_node_offsets,
                                  uint32_t row0, uint32_t n_rows, uint16_t* d_x, void* stream) {
  if (!d_feat || !d_hyp_node_offsets || !d_x) return fail(HTH_E_INVALID, "NULL argument");
  if (!n_rows) return HTH_OK;
  hipLaunchKernelGGL(k_densify, dim3(n_rows), dim3(256), 0, static_cast<hipStream_t>(stream), d_feat,
                     d_hyp_node_offsets, row0, n_rows, nullptr, nullptr, nullptr, 0u,
                     reinterpret_cast<__bf16*>(d_x));
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_densify_delta(const uint16_t* d_feat, const uint32_t* d_hyp_node_offsets,
                                        uint32_t row0, uint32_t n_rows, const uint16_t* d_parent_feat,
                                        const uint32_t* d_parent_offsets, const uint32_t* d_parent_index,
                                        uint32_t parent_context, uint16_t* d_x, void* stream) {
  if (!d_feat || !d_hyp_node_offsets || !d_parent_feat || !d_parent_offsets || !d_parent_index || !d_x)
    return fail(HTH_E_INVALID, "NULL argument");
  if (parent_context > 1) return fail(HTH_E_RANGE, "parent_context must be 0 or 1");
  if (!n_rows) return HTH_OK;
  hipLaunchKernelGGL(k_densify, dim3(n_rows), dim3(256), 0, static_cast<hipStream_t>(stream), d_feat,
                     d_hyp_node_offsets, row0, n_rows, d_parent_feat, d_parent_offsets, d_parent_index,
                     parent_context, reinterpret_cast<__bf16*>(d_x));
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_gemm_bf16(int trans_a, int trans_b, int M, int N, int K, const uint16_t* A,
                                    int lda, const uint16_t* B, int ldb, const float* bias, int relu,
                                    const uint16_t* mask, int ldm, float* c32, int ldc, uint16_t* cbf,
                                    int ldcb, void* stream) {
  if (!A || !B || (!c32 && !cbf)) return fail(HTH_E_INVALID, "NULL argument");
  if (M <= 0 || N <= 0 || K <= 0) return fail(HTH_E_RANGE, "M, N, K must be positive");
  if ((trans_a == 0 && (K % 8 || lda % 8)) || (trans_a == 1 && (M % 8 || lda % 8)) ||
      (trans_b == 0 && (N % 8 || ldb % 8)) || (trans_b == 1 && (K % 8 || ldb % 8)))
    return fail(HTH_E_INVALID, "the contiguous dimension and leading dimensions must be multiples of 8");
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) % 16)
    return fail(HTH_E_INVALID, "A and B must be 16-byte aligned");
  if (trans_a == 1 && trans_b == 1) return fail(HTH_E_UNSUPPORTED, "A^T B^T is not provided");
  GemmEpi ep{bias, relu, reinterpret_cast<const __bf16*>(mask), ldm, c32, ldc,
             reinterpret_cast<__bf16*>(cbf), ldcb};
  const dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM), block(256);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const __bf16* a = reinterpret_cast<const __bf16*>(A);
  const __bf16* b = reinterpret_cast<const __bf16*>(B);
  if (trans_a == 0 && trans_b == 0)
    hipLaunchKernelGGL((k_gemm_bf16<0, 0>), grid, block, 0, st, M, N, K, a, lda, b, ldb, ep);
  else if (trans_a == 0)
    hipLaunchKernelGGL(k_gemm_nt, grid, block, 0, st, M, N, K, a, lda, b, ldb, ep);
  else
    hipLaunchKernelGGL((k_gemm_bf16<1, 0>), grid, block, 0, st, M, N, K, a, lda, b, ldb, ep);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_head_forward(const uint16_t* h, int Bn, int Kd, const float* w, const float* bias,
                                       float* z, const float* y, float* dz, float scale, float* loss,
                                       int loss_kind, void* stream) {
  if (!h || !w || !bias || !z || (y && !dz)) return fail(HTH_E_INVALID, "NULL argument");
  if (loss_kind != 0 && loss_kind != 1) return fail(HTH_E_RANGE, "loss_kind must be 0 or 1");
  if (Bn <= 0) return HTH_OK;
  hipLaunchKernelGGL(k_head_forward, dim3((Bn + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const __bf16*>(h), Bn, Kd, w, bias, z, y, dz, scale, loss, loss_kind);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_head_score(const float* z, int Bn, float n_pos, float n_neg, const uint32_t* base,
                                     int kind, float* score, void* stream) {
  if (!z || !score) return fail(HTH_E_INVALID, "NULL argument");
  if (kind != 0 && kind != 1) return fail(HTH_E_RANGE, "kind must be 0 or 1");
  if (kind == 1 && !base) return fail(HTH_E_INVALID, "kind 1 needs the base coverage");
  if (Bn <= 0) return HTH_OK;
  hipLaunchKernelGGL(k_head_score, dim3((Bn + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream),
                     z, Bn, n_pos, n_neg, base, kind, score);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_head_backward(const uint16_t* h, int Bn, int Kd, const float* w, const float* dz,
                                        float* dw, uint16_t* dh, void* stream) {
  if (!h || !w || !dz || !dw || !dh) return fail(HTH_E_INVALID, "NULL argument");
  hipLaunchKernelGGL(k_head_backward, dim3(Kd), dim3(256), 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const __bf16*>(h), Bn, Kd, w, dz, dw, reinterpret_cast<__bf16*>(dh));
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_colsum(const void* d, int is_bf16, int M, int N, float* out, void* stream) {
  if (M < 0 || N < 0) return fail(HTH_E_RANGE, "negative matrix size");
  if (!N) return HTH_OK;
  if (!out || (M && !d)) return fail(HTH_E_INVALID, "NULL argument");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (is_bf16)
    hipLaunchKernelGGL(k_colsum<__bf16>, dim3((N + 63) / 64), dim3(256), 0, st,
                       static_cast<const __bf16*>(d), M, N, out);
  else
    hipLaunchKernelGGL(k_colsum<float>, dim3((N + 63) / 64), dim3(256), 0, st,
                       static_cast<const float*>(d), M, N, out);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_adamw(float* p, const float* g, float* m, float* v, uint16_t* pbf, size_t n,
                                float lr, float beta1, float beta2, float eps, float wd, int step,
                                void* stream) {
  if (!p || !g || !m || !v) return fail(HTH_E_INVALID, "NULL argument");
  if (step < 1) return fail(HTH_E_RANGE, "step counts from 1");
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  const unsigned g_ = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_adamw, dim3(std::max(1u, g_)), dim3(256), 0, static_cast<hipStream_t>(stream), p, g,
                     m, v, reinterpret_cast<__bf16*>(pbf), n, lr, beta1, beta2, eps, wd, c1, c2);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_transpose_bf16(const uint16_t* src, int rows, int cols, uint16_t* dst, void* stream) {
  if (!src || !dst) return fail(HTH_E_INVALID, "NULL argument");
  if (rows <= 0 || cols <= 0) return fail(HTH_E_RANGE, "rows and cols must be positive");
  if (src == dst) return fail(HTH_E_INVALID, "the transpose is not in place");
  const dim3 grid((cols + 31) / 32, (rows + 31) / 32), block(256);
  hipLaunchKernelGGL(k_transpose_bf16, grid, block, 0, static_cast<hipStream_t>(stream),
                     reinterpret_cast<const __bf16*>(src), rows, cols, reinterpret_cast<__bf16*>(dst));
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

extern "C" hth_status hth_to_bf16(const float* s, uint16_t* d, size_t n, void* stream) {
  if (!s || !d) return fail(HTH_E_INVALID, "NULL argument");
  const unsigned g_ = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_to_bf16, dim3(std::max(1u, g_)), dim3(256), 0, static_cast<hipStream_t>(stream), s,
                     reinterpret_cast<__bf16*>(d), n);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}

// Indices of the k largest scores (NaN last).  Synchronous: the radix passes
// read their histograms back.  d_work: device uint32[65536 + 2].
extern "C" hth_status hth_topk(const float* d_scores, uint32_t n, uint32_t k, uint32_t* d_idx,
                               uint32_t* d_work, void* stream) {
  if (!d_scores || !d_idx || !d_work) return fail(HTH_E_INVALID, "NULL argument");
  if (k > n) return fail(HTH_E_RANGE, "k > n");
  if (k == 0) return HTH_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint32_t prefix = 0, pmask = 0, need = k;
  std::vector<uint32_t> hist(65536);
  const unsigned grid = std::min<unsigned>((n + 255) / 256, 4096);
  for (int pass = 0; pass < 2; ++pass) {
    const uint32_t shift = pass == 0 ? 16 : 0;
    HTH_HIP(hipMemsetAsync(d_work, 0, 65536 * 4, st));
    hipLaunchKernelGGL(k_topk_hist, dim3(grid), dim3(256), 0, st, d_scores, n, shift, prefix, pmask, d_work);
    HTH_HIP(hipGetLastError());
    HTH_HIP(hipMemcpyAsync(hist.data(), d_work, 65536 * 4, hipMemcpyDeviceToHost, st));
    HTH_HIP(hipStreamSynchronize(st));
    uint32_t acc = 0, b = 65535;
    for (;; --b) {
      if (acc + hist[b] >= need) break;
      acc += hist[b];
      if (b == 0) break;
    }
    need -= acc;                   // still to take among keys whose digit == b
    prefix |= b << shift;
    pmask |= 0xFFFFu << shift;
  }
  HTH_HIP(hipMemsetAsync(d_work, 0, 8, st));
  hipLaunchKernelGGL(k_topk_collect, dim3(grid), dim3(256), 0, st, d_scores, n, prefix, need, d_idx, d_work);
  HTH_HIP(hipGetLastError());
  return HTH_OK;
}
