// Multilayer perceptron of the solve surrogate, gfx950 (MI355X): BF16 matrix
// cores (v_mfma_f32_32x32x16_bf16) with FP32 accumulation for every linear
// layer of the forward and backward pass, FP32 bias, SiLU, loss and Adam.
//
// All matrix products are "NT": C[M][N] = sum_k A[m][k] Bt[n][k], both
// operands contiguous in k, so every lane loads its MFMA operand (8 BF16
// values along k) as one 16-byte load.  The backward pass therefore keeps
// transposed copies where a product runs over the batch: activations and
// their gradients are written row-major for the next layer and, by the same
// kernel, transposed for the weight gradient.  A wave computes a 64 x 64
// tile (2 x 2 MFMA blocks), a block of four waves 128 x 128.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "radiotrace_mlp.h"
#include "rt_params.hpp"

namespace rt {
namespace mlp {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kLayers = RT_MLP_HIDDEN + 1;
static_assert(RT_MLP_OUT <= 16, "the output gradients are held 16 wide");
constexpr int kIn[kLayers] = {RT_MLP_IN, RT_MLP_WIDTH, RT_MLP_WIDTH, RT_MLP_WIDTH, RT_MLP_WIDTH};
constexpr int kOut[kLayers] = {RT_MLP_WIDTH, RT_MLP_WIDTH, RT_MLP_WIDTH, RT_MLP_WIDTH,
                               RT_MLP_OUT};

constexpr int pad16(int x) { return (x + 15) / 16 * 16; }
constexpr int64_t pad16l(int64_t x) { return (x + 15) / 16 * 16; }

// The logistic function from the hardware base-2 exponential and
// reciprocal (about 1 ulp each; e^-z overflowing to +inf gives 0, the
// limit): relative errors near 1e-7, far below the BF16 rounding (2^-9)
// that every activation then takes, and a fraction of the instructions of
// an IEEE division and the library exponential.
__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(z * -1.4426950408889634f));
}
__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

enum Epi : int {
  EPI_PLAIN = 0,         // C = acc
  EPI_OUT = 1,           // C = acc + bias
  EPI_HIDDEN_INFER = 2,  // A = bf16(silu(acc + bias))
  EPI_HIDDEN_TRAIN = 3   // C = z = acc + bias; A = bf16(silu(z)); AT = transpose of A
};

struct GemmArgs {
  const bf16* A;  // [M][lda], k contiguous
  const bf16* Bt; // [N][ldb], k contiguous
  int lda, ldb, M, N, K;  // K a multiple of 16; operands zero-padded in k up to K
  float* C;
  int ldc;
  const float* bias;
  bf16* Aout;     // [M][lda_out]
  int lda_out;
  bf16* AoutT;    // [N][ldt]; rows of the transposed copy are written up to Mpad
  int ldt, Mpad;
  // split-K (EPI_PLAIN only): block z sums k in [z kslice, (z + 1) kslice)
  // and writes its partial product to C + z M ldc; 0 = one slice
  int kslice;
};

template <int EPI>
__global__ void __launch_bounds__(256) gemm_nt_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 128 + (w >> 1) * 64;  // rows on x: batches of up to 2^24
  const int col0 = blockIdx.y * 128 + (w & 1) * 64;
  const int r = lane & 31, kh = (lane >> 5) * 8;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
  const bf16x8 zero = {};
  const bf16* pa[2];
  const bf16* pb[2];
  bool oka[2], okb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = row0 + i * 32 + r;
    oka[i] = row < g.M;
    pa[i] = g.A + (size_t)(oka[i] ? row : 0) * g.lda + kh;
    const int col = col0 + i * 32 + r;
    okb[i] = col < g.N;
    pb[i] = g.Bt + (size_t)(okb[i] ? col : 0) * g.ldb + kh;
  }
  int k0 = 0, k1 = g.K;
  float* Cout = g.C;
  if constexpr (EPI == EPI_PLAIN) {
    if (g.kslice > 0) {
      k0 = (int)blockIdx.z * g.kslice;
      k1 = min(g.K, k0 + g.kslice);
      Cout = g.C + (size_t)blockIdx.z * g.M * g.ldc;
    }
  }
  for (int k = k0; k < k1; k += 16) {
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = oka[i] ? *reinterpret_cast<const bf16x8*>(pa[i] + k) : zero;
      b[i] = okb[i] ? *reinterpret_cast<const bf16x8*>(pb[i] + k) : zero;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
  // lane holds column col0 + 32 j + (lane & 31) and, for v = 0..15, row
  // row0 + 32 i + 8 (v / 4) + 4 (lane / 32) + v % 4
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = col0 + j * 32 + r;
    if (col >= g.N) continue;
    float b = 0.0f;
    if constexpr (EPI != EPI_PLAIN) b = g.bias[col];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rb = row0 + i * 32 + q * 8 + (lane >> 5) * 4;  // first of 4 rows
        float val[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) val[u] = acc[i][j][q * 4 + u] + b;
        if constexpr (EPI == EPI_PLAIN || EPI == EPI_OUT) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (rb + u < g.M) Cout[(size_t)(rb + u) * g.ldc + col] = val[u];
        } else {
          float a[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) a[u] = silu(val[u]);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (rb + u < g.M) {
              if constexpr (EPI == EPI_HIDDEN_TRAIN) g.C[(size_t)(rb + u) * g.ldc + col] = val[u];
              g.Aout[(size_t)(rb + u) * g.lda_out + col] = (bf16)a[u];
            }
          }
          if constexpr (EPI == EPI_HIDDEN_TRAIN) {
            // transposed copy; rows beyond M (up to Mpad) are zero padding
            bf16* t = g.AoutT + (size_t)col * g.ldt + rb;
            if (rb + 3 < g.M) {
              bf16x4 pk = {(bf16)a[0], (bf16)a[1], (bf16)a[2], (bf16)a[3]};
              *reinterpret_cast<bf16x4*>(t) = pk;
            } else {
#pragma unroll
              for (int u = 0; u < 4; ++u)
                if (rb + u < g.Mpad) t[u] = (bf16)(rb + u < g.M ? a[u] : 0.0f);
            }
          }
        }
      }
  }
}

// Inference of the whole network in one launch.  A block of four waves takes
// 128 rows of the batch; their activations stay in LDS from layer to layer
// (BF16, rows padded to kActLd values so that the 32 rows a wave's lanes
// read at one k land in different banks).  Wave w computes columns 64 w ...
// 64 w + 63 of each hidden layer for all 128 rows, reading those columns of
// the layer's weights from L2 (each weight is read once per block); the
// output layer gives wave w rows 32 w ... 32 w + 31.  Every output element is
// accumulated by the same MFMA sequence over k as in gemm_nt_kernel and
// finished by the same epilogue, so the result equals the layer-by-layer
// launches bit for bit; what it saves is the round trip of every activation
// through HBM (2 x 512 MB per hidden layer at a million rows).
constexpr int kInferRows = 128;
constexpr int kActLd = RT_MLP_WIDTH + 8;
struct InferArgs {
  const bf16* wb[kLayers];    // packed weights [out][ldw]
  int ldw[kLayers];
  const float* bias[kLayers];
};

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) mlp_infer_kernel(const bf16* __restrict__ x0, InferArgs g,
                                                        int64_t B, float* __restrict__ y) {
  static_assert(RT_MLP_WIDTH == 256 && RT_MLP_HIDDEN == 4 && RT_MLP_OUT <= 32,
                "the fused inference tiles a 256-wide network");
  __shared__ bf16 act[kInferRows * kActLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 31, kh = (lane >> 5) * 8;
  const int64_t rowb = (int64_t)blockIdx.x * kInferRows;
  const bf16x8 zero = {};
  for (int h = 0; h < RT_MLP_HIDDEN; ++h) {
    const int col0 = w * 64;
    const bf16* Wl = g.wb[h];
    const int ldw = g.ldw[h];
    const bf16* wrow[2] = {Wl + (int64_t)(col0 + r) * ldw + kh,
                           Wl + (int64_t)(col0 + 32 + r) * ldw + kh};
    f32x16 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;
    if (h == 0) {
      // the 16 (padded) input features: one k step, A from the batch
      bf16x8 a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t grow = rowb + i * 32 + r;
        a[i] = grow < B ? *reinterpret_cast<const bf16x8*>(x0 + grow * 16 + kh) : zero;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(wrow[j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    } else {
      // K = 256 from the LDS activations; the weights of step k + 16 are
      // loaded before the products of step k
      bf16x8 b[2], bn[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(wrow[j]);
#pragma unroll
      for (int k = 0; k < RT_MLP_WIDTH; k += 16) {
        if (k + 16 < RT_MLP_WIDTH) {
#pragma unroll
          for (int j = 0; j < 2; ++j) bn[j] = *reinterpret_cast<const bf16x8*>(wrow[j] + k + 16);
        }
        bf16x8 a[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          a[i] = *reinterpret_cast<const bf16x8*>(act + (i * 32 + r) * kActLd + k + kh);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = bn[j];
      }
    }
    __syncthreads();  // every wave has read this layer's input
    // lane holds column col0 + 32 j + (lane & 31) and, for v = 0..15, row
    // 32 i + 8 (v / 4) + 4 (lane / 32) + v % 4
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = col0 + j * 32 + r;
      const float bj = g.bias[h][col];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rb = i * 32 + q * 8 + (lane >> 5) * 4;
#pragma unroll
          for (int u = 0; u < 4; ++u)
            act[(rb + u) * kActLd + col] = (bf16)silu(acc[i][j][q * 4 + u] + bj);
        }
    }
    __syncthreads();
  }
  // output layer: rows 32 w ... 32 w + 31, columns 0 ... 31 (RT_MLP_OUT used)
  {
    const bf16* Wl = g.wb[RT_MLP_HIDDEN];
    const int ldw = g.ldw[RT_MLP_HIDDEN];
    const bool okb = r < RT_MLP_OUT;
    f32x16 acc;
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
    for (int k = 0; k < RT_MLP_WIDTH; k += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(act + (w * 32 + r) * kActLd + k + kh);
      const bf16x8 b = okb ? *reinterpret_cast<const bf16x8*>(Wl + (int64_t)r * ldw + k + kh)
                           : zero;
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    if (okb) {
      const float bo = g.bias[RT_MLP_HIDDEN][r];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rb = w * 32 + q * 8 + (lane >> 5) * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t grow = rowb + rb + u;
          if (grow < B) y[grow * RT_MLP_OUT + r] = acc[q * 4 + u] + bo;
        }
      }
    }
  }
}

// Features [B][5] FP32 -> x0 [B][16] BF16 (zero-padded) and, for training,
// x0T [16][Bp] (zero beyond B).
__global__ void features_kernel(const float* __restrict__ x, int64_t B, int64_t Bp,
                                bf16* __restrict__ x0, bf16* __restrict__ x0T) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bp) return;
  for (int k = 0; k < 16; ++k) {
    const float v = (b < B && k < RT_MLP_IN) ? x[b * RT_MLP_IN + k] : 0.0f;
    if (b < B) x0[b * 16 + k] = (bf16)v;
    if (x0T) x0T[(int64_t)k * Bp + b] = (bf16)v;
  }
}

// Loss of the header and its gradient w.r.t. the outputs; dY [B][16] and
// dYT [16][Bp] in BF16 (zero padding), per-block partial sums of the loss.
// Labels per row: existence of families 0, 1, then several roots in 0, 1.
__global__ void __launch_bounds__(256) loss_kernel(const float* __restrict__ y,
                                                   const float* __restrict__ t,
                                                   const float* __restrict__ m, int64_t B,
                                                   int64_t Bp, bf16* __restrict__ dY,
                                                   bf16* __restrict__ dYT,
                                                   float* __restrict__ partial) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.0f;
  if (b < Bp) {
    float d[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) d[q] = 0.0f;
    if (b < B) {
      const float invB = 1.0f / (float)B;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const float mf = m[b * RT_MLP_LABELS + f];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float e = y[b * RT_MLP_OUT + 4 * f + q] - t[b * RT_MLP_TARGETS + 4 * f + q];
          l += mf * e * e;
          d[4 * f + q] = 2.0f * mf * e * invB;
        }
        const float z = y[b * RT_MLP_OUT + 8 + f];
        // log(1 + e^z) - m z, evaluated without overflow
        l += fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))) - mf * z;
        d[8 + f] = (1.0f / (1.0f + expf(-z)) - mf) * invB;
        const float rf = m[b * RT_MLP_LABELS + 2 + f];
        const float zr = y[b * RT_MLP_OUT + 10 + f];
        l += fmaxf(zr, 0.0f) + log1pf(expf(-fabsf(zr))) - rf * zr;
        d[10 + f] = (1.0f / (1.0f + expf(-zr)) - rf) * invB;
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) dY[b * 16 + q] = (bf16)d[q];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) dYT[(int64_t)q * Bp + b] = (bf16)d[q];
  }
  __shared__ float red[256];
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) loss_final_kernel(const float* __restrict__ partial,
                                                         int n, int64_t B, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)B;
}

// dZ = dA * silu'(Z): [B][256] BF16 and transposed [256][Bp], through a
// 32 x 32 LDS tile so that both writes are coalesced.
__global__ void __launch_bounds__(256) silu_back_kernel(const float* __restrict__ dA,
                                                        const float* __restrict__ Z, int64_t B,
                                                        int64_t Bp, bf16* __restrict__ dZ,
                                                        bf16* __restrict__ dZT) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t b0 = (int64_t)blockIdx.x * 32;
  const int j0 = blockIdx.y * 32;
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t b = b0 + yy;
    const int j = j0 + tx;
    float v = 0.0f;
    if (b < B) {
      const int64_t i = b * RT_MLP_WIDTH + j;
      v = dA[i] * silu_grad(Z[i]);
      dZ[i] = (bf16)v;
    }
    tile[yy][tx] = v;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int j = j0 + yy;
    const int64_t b = b0 + tx;
    if (b < Bp) dZT[(int64_t)j * Bp + b] = (bf16)tile[tx][yy];
  }
}

// out[r] = sum over the n columns of row r of a BF16 matrix (bias gradients):
// 16-byte loads of 8 values (rows start 16-byte aligned: ld a multiple of 8),
// then the wave sums and the four waves' sums.
__global__ void __launch_bounds__(256) rowsum_kernel(const bf16* __restrict__ X, int64_t ld,
                                                     int64_t n, float* __restrict__ out) {
  __shared__ float red[4];
  const bf16* row = X + (int64_t)blockIdx.x * ld;
  float s = 0.0f;
  const int64_t n8 = n / 8;
  for (int64_t i = threadIdx.x; i < n8; i += 256) {
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(row + 8 * i);
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (float)v[u];
  }
  for (int64_t i = 8 * n8 + threadIdx.x; i < n; i += 256) s += (float)row[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// out[i] = sum over s < S of part[s n + i]: the slices of a split-K product,
// added in slice order (the result does not depend on the launch).
__global__ void __launch_bounds__(256) splitk_sum_kernel(const float* __restrict__ part, int S,
                                                         int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = part[i];
  int z = 1;
  // eight slices' loads in flight, added in slice order
  for (; z + 8 <= S; z += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(z + u) * n + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; z < S; ++z) acc += part[(int64_t)z * n + i];
  out[i] = acc;
}

// W [N][K] FP32 -> Wb [N][Kp] BF16 and (optional) WbT [K][Np] BF16, zero padded.
__global__ void pack_layer_kernel(const float* __restrict__ W, int N, int K, bf16* __restrict__ Wb,
                                  int Kp, bf16* __restrict__ WbT, int Np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)N * Kp) {
    const int n = (int)(i / Kp), k = (int)(i % Kp);
    Wb[i] = (bf16)(k < K ? W[(int64_t)n * K + k] : 0.0f);
  }
  if (WbT && i < (int64_t)K * Np) {
    const int k = (int)(i / Np), n = (int)(i % Np);
    WbT[i] = (bf16)(n < N ? W[(int64_t)n * K + k] : 0.0f);
  }
}

__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ---------------------------------------------------------------------------
// Host side: parameter offsets and workspace layout.
struct Offsets {
  int64_t w[kLayers], b[kLayers], total;
};
Offsets param_offsets() {
  Offsets o;
  int64_t off = 0;
  for (int l = 0; l < kLayers; ++l) {
    o.w[l] = off;
    off += (int64_t)kIn[l] * kOut[l];
    o.b[l] = off;
    off += kOut[l];
  }
  o.total = off;
  return o;
}

// Packed weights: Wb_l [out][pad16(in)] for every layer, WbT_l [in][pad16(out)]
// for layers 1..4; then per-batch buffers.
struct Layout {
  bf16* wb[kLayers];
  bf16* wbt[kLayers];
  bf16 *x0, *x0T;
  float* z[RT_MLP_HIDDEN];
  bf16* a[RT_MLP_HIDDEN];
  bf16* aT[RT_MLP_HIDDEN];
  float* y;
  bf16 *dy, *dyT;
  float* dA;
  bf16 *dz, *dzT;
  float* partial;
  float* splitk;  // kMaxSlices partial products of up to 256 x 256
  size_t bytes;
};

// Weight gradients sum over the batch: split into slices of at least 256
// rows (16 matrix-core steps), at most kMaxSlices of them, so that a
// 256 x 256 gradient keeps 4 x slices workgroups busy instead of 4.
constexpr int kMaxSlices = 32;
constexpr int kMinSliceK = 256;

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

// Layout for batch B; training adds the backward buffers.  With base NULL
// only the size is computed.
Layout layout(char* base, int64_t B, bool training) {
  Layout L;
  memset(&L, 0, sizeof L);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  for (int l = 0; l < kLayers; ++l)
    L.wb[l] = reinterpret_cast<bf16*>(take((size_t)kOut[l] * pad16(kIn[l]) * 2));
  for (int l = 1; l < kLayers; ++l)
    L.wbt[l] = reinterpret_cast<bf16*>(take((size_t)kIn[l] * pad16(kOut[l]) * 2));
  off = align_up(off + 4096);  // the packed weights end here for every batch size
  const int64_t Bp = pad16l(B);
  L.x0 = reinterpret_cast<bf16*>(take((size_t)B * 16 * 2));
  if (!training) {
    L.a[0] = reinterpret_cast<bf16*>(take((size_t)B * RT_MLP_WIDTH * 2));
    L.a[1] = reinterpret_cast<bf16*>(take((size_t)B * RT_MLP_WIDTH * 2));
  } else {
    L.x0T = reinterpret_cast<bf16*>(take((size_t)16 * Bp * 2));
    for (int h = 0; h < RT_MLP_HIDDEN; ++h) {
      L.z[h] = reinterpret_cast<float*>(take((size_t)B * RT_MLP_WIDTH * 4));
      L.a[h] = reinterpret_cast<bf16*>(take((size_t)B * RT_MLP_WIDTH * 2));
      L.aT[h] = reinterpret_cast<bf16*>(take((size_t)RT_MLP_WIDTH * Bp * 2));
    }
    L.y = reinterpret_cast<float*>(take((size_t)B * RT_MLP_OUT * 4));
    L.dy = reinterpret_cast<bf16*>(take((size_t)B * 16 * 2));
    L.dyT = reinterpret_cast<bf16*>(take((size_t)16 * Bp * 2));
    L.dA = reinterpret_cast<float*>(take((size_t)B * RT_MLP_WIDTH * 4));
    L.dz = reinterpret_cast<bf16*>(take((size_t)B * RT_MLP_WIDTH * 2));
    L.dzT = reinterpret_cast<bf16*>(take((size_t)RT_MLP_WIDTH * Bp * 2));
    L.partial = reinterpret_cast<float*>(take((size_t)((Bp + 255) / 256) * 4));
    L.splitk = reinterpret_cast<float*>(
        take((size_t)kMaxSlices * RT_MLP_WIDTH * RT_MLP_WIDTH * 4));
  }
  L.bytes = off;
  return L;
}

template <int EPI>
hipError_t gemm(const GemmArgs& g, hipStream_t s) {
  const unsigned nz = g.kslice > 0 ? (unsigned)((g.K + g.kslice - 1) / g.kslice) : 1u;
  dim3 grid((unsigned)((g.M + 127) / 128), (unsigned)((g.N + 127) / 128), nz);
  hipLaunchKernelGGL((gemm_nt_kernel<EPI>), grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// Weight gradient C[M][N] (M, N <= 256) = sum over the K batch rows, as a
// split-K product into the slice buffer and a slice sum into C.
hipError_t weight_grad(GemmArgs g, float* slices, hipStream_t s) {
  int S = std::min(kMaxSlices, std::max(1, g.K / kMinSliceK));
  const int ks = (g.K / 16 + S - 1) / S * 16;  // a multiple of 16
  S = (g.K + ks - 1) / ks;
  float* C = g.C;
  g.kslice = ks;
  g.C = slices;
  hipError_t e = gemm<EPI_PLAIN>(g, s);
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)g.M * g.ldc;
  hipLaunchKernelGGL(splitk_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     slices, S, n, C);
  return hipGetLastError();
}

GemmArgs args(const bf16* A, int lda, const bf16* Bt, int ldb, int M, int N, int K, float* C,
              int ldc) {
  GemmArgs g;
  memset(&g, 0, sizeof g);
  g.A = A;
  g.lda = lda;
  g.Bt = Bt;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.C = C;
  g.ldc = ldc;
  return g;
}

}  // namespace mlp
}  // namespace rt

#define HIP_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      rt::set_last_error("%s: %s", #expr, hipGetErrorString(e_));             \
      return RT_ERR_DEVICE;                                                   \
    }                                                                         \
  } while (0)

namespace {
rt_status check_ws(const void* ws, size_t bytes, int64_t batch, bool training) {
  using namespace rt;
  if (!ws) {
    set_last_error("null workspace");
    return RT_ERR_INVALID_ARG;
  }
  if (batch < 1 || batch > ((int64_t)1 << 24)) {
    set_last_error("batch must be 1..2^24");
    return RT_ERR_INVALID_ARG;
  }
  const size_t need = mlp::layout(nullptr, batch, training).bytes;
  if (bytes < need) {
    set_last_error("workspace of %zu bytes < %zu needed for batch %lld%s", bytes, need,
                   (long long)batch, training ? " (training)" : "");
    return RT_ERR_INVALID_ARG;
  }
  return RT_OK;
}
}  // namespace

extern "C" int64_t rt_mlp_param_count(void) { return rt::mlp::param_offsets().total; }

extern "C" rt_status rt_mlp_workspace_bytes(int64_t batch, int32_t training, size_t* bytes) {
  if (!bytes || batch < 1 || batch > ((int64_t)1 << 24)) {
    rt::set_last_error("need bytes != NULL and 1 <= batch <= 2^24");
    return RT_ERR_INVALID_ARG;
  }
  *bytes = rt::mlp::layout(nullptr, batch, training != 0).bytes;
  return RT_OK;
}

extern "C" rt_status rt_mlp_pack(const float* params, void* ws, size_t bytes, void* stream) {
  using namespace rt::mlp;
  rt_status st = check_ws(ws, bytes, 1, false);
  if (st != RT_OK) return st;
  if (!params) {
    rt::set_last_error("null params");
    return RT_ERR_INVALID_ARG;
  }
  const Offsets o = param_offsets();
  const Layout L = layout(static_cast<char*>(ws), 1, false);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int l = 0; l < kLayers; ++l) {
    const int N = kOut[l], K = kIn[l], Kp = pad16(K), Np = pad16(N);
    const int64_t n = std::max((int64_t)N * Kp, (int64_t)K * Np);
    hipLaunchKernelGGL(pack_layer_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       params + o.w[l], N, K, L.wb[l], Kp, L.wbt[l], Np);
    HIP_TRY(hipGetLastError());
  }
  return RT_OK;
}

extern "C" rt_status rt_mlp_forward(const float* params, const float* x, int64_t B, float* y,
                                    void* ws, size_t bytes, void* stream) {
  using namespace rt::mlp;
  rt_status st = check_ws(ws, bytes, B, false);
  if (st != RT_OK) return st;
  if (!params || !x || !y) {
    rt::set_last_error("null params, x or y");
    return RT_ERR_INVALID_ARG;
  }
  const Offsets o = param_offsets();
  const Layout L = layout(static_cast<char*>(ws), B, false);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, x, B,
                     B, L.x0, (bf16*)nullptr);
  HIP_TRY(hipGetLastError());
  InferArgs g;
  for (int l = 0; l < kLayers; ++l) {
    g.wb[l] = L.wb[l];
    g.ldw[l] = pad16(kIn[l]);
    g.bias[l] = params + o.b[l];
  }
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)((B + kInferRows - 1) / kInferRows)),
                     dim3(256), 0, s, L.x0, g, B, y);
  HIP_TRY(hipGetLastError());
  return RT_OK;
}

extern "C" rt_status rt_mlp_forward_layers(const float* params, const float* x, int64_t B,
                                           float* y, void* ws, size_t bytes, void* stream) {
  using namespace rt::mlp;
  rt_status st = check_ws(ws, bytes, B, false);
  if (st != RT_OK) return st;
  if (!params || !x || !y) {
    rt::set_last_error("null params, x or y");
    return RT_ERR_INVALID_ARG;
  }
  const Offsets o = param_offsets();
  const Layout L = layout(static_cast<char*>(ws), B, false);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, x, B,
                     B, L.x0, (bf16*)nullptr);
  HIP_TRY(hipGetLastError());
  const int M = (int)B, W = RT_MLP_WIDTH;
  const bf16* in = L.x0;
  int ld_in = 16, K = 16;
  for (int h = 0; h < RT_MLP_HIDDEN; ++h) {
    bf16* out = L.a[h & 1];
    GemmArgs g = args(in, ld_in, L.wb[h], pad16(kIn[h]), M, W, K, nullptr, 0);
    g.bias = params + o.b[h];
    g.Aout = out;
    g.lda_out = W;
    HIP_TRY(gemm<EPI_HIDDEN_INFER>(g, s));
    in = out;
    ld_in = W;
    K = W;
  }
  GemmArgs g = args(in, W, L.wb[4], W, M, RT_MLP_OUT, W, y, RT_MLP_OUT);
  g.bias = params + o.b[4];
  HIP_TRY(gemm<EPI_OUT>(g, s));
  return RT_OK;
}

extern "C" rt_status rt_mlp_gradients(const float* params, const float* x, const float* t,
                                      const float* m, int64_t B, float* grad, float* loss,
                                      void* ws, size_t bytes, void* stream) {
  using namespace rt::mlp;
  rt_status st = check_ws(ws, bytes, B, true);
  if (st != RT_OK) return st;
  if (!params || !x || !t || !m || !grad || !loss) {
    rt::set_last_error("null params, x, targets, mask, grad or loss");
    return RT_ERR_INVALID_ARG;
  }
  const Offsets o = param_offsets();
  const Layout L = layout(static_cast<char*>(ws), B, true);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t Bp = pad16l(B);
  const int M = (int)B, W = RT_MLP_WIDTH, Kb = (int)Bp;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((Bp + 255) / 256)), dim3(256), 0, s, x, B,
                     Bp, L.x0, L.x0T);
  HIP_TRY(hipGetLastError());
  // forward, keeping pre-activations and transposed activations
  const bf16* in = L.x0;
  int ld_in = 16, K = 16;
  for (int h = 0; h < RT_MLP_HIDDEN; ++h) {
    GemmArgs g = args(in, ld_in, L.wb[h], pad16(kIn[h]), M, W, K, L.z[h], W);
    g.bias = params + o.b[h];
    g.Aout = L.a[h];
    g.lda_out = W;
    g.AoutT = L.aT[h];
    g.ldt = Kb;
    g.Mpad = Kb;
    HIP_TRY(gemm<EPI_HIDDEN_TRAIN>(g, s));
    in = L.a[h];
    ld_in = W;
    K = W;
  }
  {
    GemmArgs g = args(in, W, L.wb[4], W, M, RT_MLP_OUT, W, L.y, RT_MLP_OUT);
    g.bias = params + o.b[4];
    HIP_TRY(gemm<EPI_OUT>(g, s));
  }
  // loss and output gradient
  const int nblk = (int)((Bp + 255) / 256);
  hipLaunchKernelGGL(loss_kernel, dim3((unsigned)nblk), dim3(256), 0, s, L.y, t, m, B, Bp, L.dy,
                     L.dyT, L.partial);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, s, L.partial, nblk, B, loss);
  HIP_TRY(hipGetLastError());
  // output layer: db4, dW4 = dY^T a3, dA3 = dY W4
  hipLaunchKernelGGL(rowsum_kernel, dim3(RT_MLP_OUT), dim3(256), 0, s, L.dyT, Bp, Bp,
                     grad + o.b[4]);
  HIP_TRY(hipGetLastError());
  HIP_TRY(weight_grad(args(L.dyT, Kb, L.aT[3], Kb, RT_MLP_OUT, W, Kb, grad + o.w[4], W), L.splitk,
                      s));
  HIP_TRY(gemm<EPI_PLAIN>(args(L.dy, 16, L.wbt[4], 16, M, W, 16, L.dA, W), s));
  for (int h = RT_MLP_HIDDEN - 1; h >= 0; --h) {
    dim3 tg((unsigned)((Bp + 31) / 32), W / 32);
    hipLaunchKernelGGL(silu_back_kernel, tg, dim3(256), 0, s, L.dA, L.z[h], B, Bp, L.dz, L.dzT);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(rowsum_kernel, dim3(W), dim3(256), 0, s, L.dzT, Bp, Bp, grad + o.b[h]);
    HIP_TRY(hipGetLastError());
    const bf16* prevT = h > 0 ? L.aT[h - 1] : L.x0T;
    const int n_in = kIn[h];
    HIP_TRY(weight_grad(args(L.dzT, Kb, prevT, Kb, W, n_in, Kb, grad + o.w[h], n_in), L.splitk,
                        s));
    if (h > 0) HIP_TRY(gemm<EPI_PLAIN>(args(L.dz, W, L.wbt[h], W, M, W, W, L.dA, W), s));
  }
  return RT_OK;
}

extern "C" rt_status rt_mlp_adam(float* params, float* m, float* v, const float* grad,
                                 int64_t step, const rt_adam* hp, void* ws, size_t bytes,
                                 void* stream) {
  using namespace rt::mlp;
  if (!params || !m || !v || !grad || !hp || step < 1) {
    rt::set_last_error("null argument or step < 1");
    return RT_ERR_INVALID_ARG;
  }
  if (!(hp->lr > 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) ||
      !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) || !(hp->eps > 0.0f)) {
    rt::set_last_error("need lr > 0, 0 <= beta < 1, eps > 0");
    return RT_ERR_INVALID_ARG;
  }
  const int64_t n = param_offsets().total;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)hp->beta1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)hp->beta2, (double)step)));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, m,
                     v, grad, n, hp->lr, hp->beta1, hp->beta2, hp->eps, c1, c2);
  HIP_TRY(hipGetLastError());
  return rt_mlp_pack(params, ws, bytes, stream);
}
