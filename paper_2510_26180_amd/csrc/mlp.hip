// Learned initial guess: an MLP xi -> coarse-grid states of every slice, trained and
// evaluated with BF16 MFMA GEMMs (32x32x16, FP32 accumulation) on gfx950.
//
// It replaces the gPC map of Algorithm 3 step 6 by a network fitted to solutions that
// the method itself produced; the parareal iteration (Algorithm 2) is unchanged.
//   pre1 = X W1 + b1, h1 = GELU(pre1);  pre2 = h1 W2 + b2, h2 = GELU(pre2);
//   Y = h2 W3 + b3;  loss = mean((Y - T)^2) over z-scored targets T;  Adam with FP32
//   master weights.  GELU is the exact x Phi(x).
// BF16 rounding points (round to nearest even): the GEMM operands X, W1..W3, h1, h2,
// dY, dpre2, dpre1.  Bias gradients and GELU derivatives use the FP32 values.
// Grid transfer: bilinear interpolation with zero boundary values between the n x n
// grid (h = 1/(n+1)) and the nc x nc grid (H = 1/(nc+1)), evaluated at the nodes of
// the other grid.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <vector>

#include "common.h"

typedef unsigned short kc_bf16;

struct klecgc_mlp {
  int32_t n_in = 0, in_pad = 0, hidden = 0;
  int64_t n_out = 0, n_params = 0;
  float* w = nullptr;     // FP32 masters, flat [W1 b1 W2 b2 W3 b3], W row-major [in][out]
  float* m = nullptr;     // Adam first moments
  float* v = nullptr;     // Adam second moments
  float* g = nullptr;     // gradient of the last batch (same layout)
  kc_bf16* wb = nullptr;  // BF16 copies: W1 [in_pad][H] (rows >= n_in zero), W2, W3
  float* mean = nullptr;  // target normalisation [n_out]
  float* stdv = nullptr;
  int64_t t = 0;          // Adam step count
  int cap_b = 0;          // rows the work buffer holds
  void* ws = nullptr;
  size_t ws_bytes = 0;
};

namespace kc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ kc_bf16 f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (kc_bf16)((u >> 16) | 0x40);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                         // nearest, ties to even
  return (kc_bf16)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2 };
constexpr int GBM = 64, GBN = 64, GBK = 32, LDK = GBK + 8;

// C[z] = op(A) op(B) over k in [z kchunk, (z+1) kchunk), z = blockIdx.z (split-K partials;
// a single split when kchunk >= K), optional + bias and GELU (then also a BF16 copy).
//   !TA: A [M][K] (lda)   TA: A stored [K][M]      !TB: B [K][N]   TB: B stored [N][K]
// 256 threads = 4 waves, each owning one 32x32 quarter of the 64x64 tile.  Operand
// layout of v_mfma_f32_32x32x16_bf16 (checked on gfx950): A lane l holds row l%32,
// k = 8(l/32)+e; B lane l holds column l%32, k = 8(l/32)+e; result element e of lane
// l is row 8(e/4)+4(l/32)+e%4, column l%32.  LDS keeps both tiles k-contiguous
// ([row][k], [col][k]) so each lane's eight k-values are one 16-byte read.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, int kchunk, const kc_bf16* __restrict__ A,
                                                        int lda, const kc_bf16* __restrict__ B, int ldb,
                                                        float* __restrict__ C, int ldc, const float* __restrict__ bias,
                                                        kc_bf16* __restrict__ Cb, int ldcb) {
  __shared__ __attribute__((aligned(16))) kc_bf16 As[GBM][LDK];
  __shared__ __attribute__((aligned(16))) kc_bf16 Bs[GBN][LDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int row0 = blockIdx.y * GBM, col0 = blockIdx.x * GBN;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  C += (int64_t)blockIdx.z * M * ldc;
  const bool avec = (lda & 7) == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
  const bool bvec = (ldb & 7) == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  floatx16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += GBK) {
    if (!TA) {  // 64 rows x 4 chunks of 8 k
      const int r = tid >> 2, kc8 = (tid & 3) * 8;
      const int gi = row0 + r, gk = k0 + kc8;
      uint4 q = {0, 0, 0, 0};
      if (avec && gi < M && gk + 7 < ke) {
        q = *reinterpret_cast<const uint4*>(A + (int64_t)gi * lda + gk);
      } else {
        kc_bf16 t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = (gi < M && gk + e < ke) ? A[(int64_t)gi * lda + gk + e] : (kc_bf16)0;
        q = *reinterpret_cast<uint4*>(t);
      }
      *reinterpret_cast<uint4*>(&As[r][kc8]) = q;
    } else {    // 32 k x 8 chunks of 8 rows, transposed into As[row][k]
      const int k = tid >> 3, r8 = (tid & 7) * 8;
      const int gk = k0 + k, gi = row0 + r8;
      kc_bf16 t[8];
      if (avec && gk < ke && gi + 7 < M) {
        *reinterpret_cast<uint4*>(t) = *reinterpret_cast<const uint4*>(A + (int64_t)gk * lda + gi);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = (gk < ke && gi + e < M) ? A[(int64_t)gk * lda + gi + e] : (kc_bf16)0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) As[r8 + e][k] = t[e];
    }
    if (TB) {   // 64 columns x 4 chunks of 8 k
      const int c = tid >> 2, kc8 = (tid & 3) * 8;
      const int gj = col0 + c, gk = k0 + kc8;
      uint4 q = {0, 0, 0, 0};
      if (bvec && gj < N && gk + 7 < ke) {
        q = *reinterpret_cast<const uint4*>(B + (int64_t)gj * ldb + gk);
      } else {
        kc_bf16 t[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = (gj < N && gk + e < ke) ? B[(int64_t)gj * ldb + gk + e] : (kc_bf16)0;
        q = *reinterpret_cast<uint4*>(t);
      }
      *reinterpret_cast<uint4*>(&Bs[c][kc8]) = q;
    } else {    // 32 k x 8 chunks of 8 columns, transposed into Bs[col][k]
      const int k = tid >> 3, c8 = (tid & 7) * 8;
      const int gk = k0 + k, gj = col0 + c8;
      kc_bf16 t[8];
      if (bvec && gk < ke && gj + 7 < N) {
        *reinterpret_cast<uint4*>(t) = *reinterpret_cast<const uint4*>(B + (int64_t)gk * ldb + gj);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = (gk < ke && gj + e < N) ? B[(int64_t)gk * ldb + gj + e] : (kc_bf16)0;
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[c8 + e][k] = t[e];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; kk += 16) {
      const int ko = kk + 8 * (lane >> 5);
      const bf16x8 a = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&As[wr + (lane & 31)][ko]));
      const bf16x8 b = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&Bs[wc + (lane & 31)][ko]));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int gj = col0 + wc + (lane & 31);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int gi = row0 + wr + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
    if (gi < M && gj < N) {
      float v = acc[e];
      if (EPI != EPI_STORE) v += bias[gj];
      C[(int64_t)gi * ldc + gj] = v;
      if (EPI == EPI_BIAS_GELU) Cb[(int64_t)gi * ldcb + gj] = f2bf(gelu_f(v));
    }
  }
}

// C[i] = sum_z P[z][i], i < total (the split-K partials)
__global__ void splitk_reduce_kernel(const float* __restrict__ P, int S, int64_t total, float* __restrict__ C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += P[(int64_t)z * total + i];
    C[i] = s;
  }
}

// Training counters in device memory, so that one epoch of steps can be replayed from a
// captured graph: t = Adam steps taken before the current one, ep = epoch of this call.
struct TrainCtr {
  int64_t t;
  int64_t ep;
};

// row of mini-batch entry b: perm[ep n + off + b] with a permutation, else off + b
__device__ __forceinline__ int64_t batch_row(const int32_t* perm, const TrainCtr* ctr, int64_t n, int64_t off, int b) {
  return perm ? (int64_t)perm[ctr->ep * n + off + b] : off + b;
}

// Xb[b][0..in_pad) = bf16(xi[row(b)][..]), zero padded
__global__ void gather_x_kernel(const double* __restrict__ xi, const int32_t* __restrict__ perm,
                                const TrainCtr* __restrict__ ctr, int64_t n_rows, int64_t off, int B, int n_in,
                                int in_pad, kc_bf16* __restrict__ Xb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)B * in_pad;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / in_pad), c = (int)(i % in_pad);
    const int64_t src = batch_row(perm, ctr, n_rows, off, b);
    Xb[i] = c < n_in ? f2bf((float)xi[src * n_in + c]) : (kc_bf16)0;
  }
}

// flag[0] = 1 if some perm entry lies outside [0, n)
__global__ void check_perm_kernel(const int32_t* __restrict__ perm, int64_t total, int32_t n, int* __restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    if (perm[i] < 0 || perm[i] >= n) *flag = 1;
}

// dY = scale (Y - T) in FP32 and BF16, T row = Tg[row(b)]; the block's sum of squares goes
// to part[block] (summed in a fixed order by loss_reduce_kernel: no contended atomics).
// grid (x blocks over columns, B rows), 256 threads.
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ Tg,
                                                       const int32_t* __restrict__ perm,
                                                       const TrainCtr* __restrict__ ctr, int64_t n_rows,
                                                       int64_t off, int64_t O, float scale, float* __restrict__ dY,
                                                       kc_bf16* __restrict__ dYb, double* __restrict__ part) {
  __shared__ double wsum[4];
  const int b = blockIdx.y;
  const int64_t src = batch_row(perm, ctr, n_rows, off, b);
  const float* y = Y + (int64_t)b * O;
  const float* t = Tg + src * O;
  double s = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < O; j += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[j] - t[j];
    s += (double)d * d;
    const float gv = scale * d;
    dY[(int64_t)b * O + j] = gv;
    dYb[(int64_t)b * O + j] = f2bf(gv);
  }
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// *loss += sum of part[0..count) (one work-group of 256 threads, fixed order)
__global__ __launch_bounds__(256) void loss_reduce_kernel(const double* __restrict__ part, int64_t count,
                                                          double* __restrict__ loss) {
  __shared__ double wsum[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) s += part[i];
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss += wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// dpre = dH * GELU'(pre), FP32 and BF16
__global__ void gelu_bwd_kernel(const float* __restrict__ dH, const float* __restrict__ pre, int64_t total,
                                float* __restrict__ dpre, kc_bf16* __restrict__ dpreb) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const float gv = dH[i] * gelu_grad_f(pre[i]);
    dpre[i] = gv;
    dpreb[i] = f2bf(gv);
  }
}

// db[j] = sum_i D[i][j]: 64 columns per work-group, the rows split over 16 slices of
// threads and summed by a fixed LDS tree (deterministic; many loads in flight per column)
__global__ __launch_bounds__(1024) void colsum_kernel(const float* __restrict__ D, int rows, int64_t cols,
                                                      float* __restrict__ db) {
  __shared__ float acc[16][64];
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + c;
  float s = 0.f;
  if (j < cols)
    for (int i = r0; i < rows; i += 16) s += D[(int64_t)i * cols + j];
  acc[r0][c] = s;
  __syncthreads();
  for (int h = 8; h >= 1; h >>= 1) {
    if (r0 < h) acc[r0][c] += acc[r0 + h][c];
    __syncthreads();
  }
  if (r0 == 0 && j < cols) db[j] = acc[0][c];
}

// Adam on the FP32 masters; the BF16 copies of the weight blocks are refreshed in the
// same pass (W1 keeps its row-major index, its padding rows are never touched).
struct AdamSeg {
  int64_t oW2, ob2, oW3, ob3, bW2, bW3;
};
// Step t+1 with bias corrections c1 = 1 - b1^(t+1), c2 = 1 - b2^(t+1) and the epoch's learning
// rate lr0 (lr_final/lr0)^(ep/(epochs-1)) (constant lr0 if lr_final <= 0), read from ctr.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t total, float lr0, float lr_final, int epochs, float b1,
                            float b2, float eps, const TrainCtr* __restrict__ ctr, int64_t nW1, AdamSeg sg,
                            kc_bf16* __restrict__ wb) {
  const double t = (double)(ctr->t + 1);
  const float c1 = (float)(1.0 - pow((double)b1, t));
  const float c2 = (float)(1.0 - pow((double)b2, t));
  const float lr = (lr_final > 0.f && epochs > 1)
                       ? (float)(lr0 * pow((double)lr_final / lr0, (double)ctr->ep / (epochs - 1)))
                       : lr0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (i < nW1)
      wb[i] = f2bf(wi);
    else if (i >= sg.oW2 && i < sg.ob2)
      wb[sg.bW2 + (i - sg.oW2)] = f2bf(wi);
    else if (i >= sg.oW3 && i < sg.ob3)
      wb[sg.bW3 + (i - sg.oW3)] = f2bf(wi);
  }
}

__global__ void step_kernel(TrainCtr* __restrict__ ctr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctr->t += 1;
}

// end of an epoch: record its mean loss, reset the accumulator, advance the epoch
__global__ void epoch_end_kernel(TrainCtr* __restrict__ ctr, double* __restrict__ loss, double* __restrict__ hist,
                                 double scale) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hist[ctr->ep] = *loss * scale;
    *loss = 0.0;
    ctr->ep += 1;
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t total, kc_bf16* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = f2bf(x[i]);
}

__global__ void fill_kernel(float* __restrict__ x, int64_t total, float val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = val;
}

// per-output mean and standard deviation over n rows (std 0 -> 1), then Y := (Y - mu)/sd
__global__ void zscore_kernel(float* __restrict__ Y, int64_t n, int64_t cols, float* __restrict__ mean,
                              float* __restrict__ stdv) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cols; j += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += Y[i * cols + j];
    const double mu = s / (double)n;
    double s2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double d = Y[i * cols + j] - mu;
      s2 += d * d;
    }
    double sd = sqrt(s2 / (double)n);
    if (!(sd > 0.0)) sd = 1.0;
    mean[j] = (float)mu;
    stdv[j] = (float)sd;
    for (int64_t i = 0; i < n; ++i) Y[i * cols + j] = (float)((Y[i * cols + j] - mu) / sd);
  }
}

// linear-interpolation stencil: node q of a grid with nt interior nodes on (0,1) lies at
// s = x_q (nf + 1) - 1 in units of the nf-node grid; weights (1-t, t) on nodes i0, i0+1
__device__ __forceinline__ void lin_weights(int q, int nt, int nf, int& i0, double& t) {
  const double x = (q + 1.0) / (nt + 1.0);
  const double s = x * (nf + 1.0) - 1.0;
  i0 = (int)floor(s);
  t = s - i0;
}

// Yc[r][Q] = bilinear interpolant of U[r][:] (n x n, x fastest) at coarse node Q
__global__ void restrict_kernel(const double* __restrict__ U, int n, int nc, int64_t R, float* __restrict__ Yc) {
  const int64_t r = blockIdx.y;
  const int Q = blockIdx.x * blockDim.x + threadIdx.x;
  if (Q >= nc * nc || r >= R) return;
  int ix, iy;
  double tx, ty;
  lin_weights(Q % nc, nc, n, ix, tx);
  lin_weights(Q / nc, nc, n, iy, ty);
  const double* u = U + r * (int64_t)n * n;
  auto at = [&](int i, int j) -> double { return (i >= 0 && i < n && j >= 0 && j < n) ? u[(int64_t)j * n + i] : 0.0; };
  const double val = (1 - ty) * ((1 - tx) * at(ix, iy) + tx * at(ix + 1, iy)) +
                     ty * ((1 - tx) * at(ix, iy + 1) + tx * at(ix + 1, iy + 1));
  Yc[r * (int64_t)nc * nc + Q] = (float)val;
}

// U[r][p] = bilinear interpolant at fine node p of the de-normalised coarse field
// mu + sd * Yz[r][:] (r = m N + s; mean and sd of slice s)
__global__ void prolong_kernel(const float* __restrict__ Yz, const float* __restrict__ mean,
                               const float* __restrict__ stdv, int n, int nc, int N, int64_t r0, int64_t R,
                               double* __restrict__ U) {
  const int64_t r = blockIdx.y;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= (int64_t)n * n || r >= R) return;
  const int s = (int)((r0 + r) % N);
  const int64_t Oc = (int64_t)nc * nc;
  const float* y = Yz + r * Oc;
  const float* mu = mean + s * Oc;
  const float* sd = stdv + s * Oc;
  int ix, iy;
  double tx, ty;
  lin_weights((int)(p % n), n, nc, ix, tx);
  lin_weights((int)(p / n), n, nc, iy, ty);
  auto at = [&](int a, int b) -> double {
    if (a < 0 || a >= nc || b < 0 || b >= nc) return 0.0;
    const int64_t q = (int64_t)b * nc + a;
    return (double)y[q] * (double)sd[q] + (double)mu[q];
  };
  U[r * (int64_t)n * n + p] = (1 - ty) * ((1 - tx) * at(ix, iy) + tx * at(ix + 1, iy)) +
                              ty * ((1 - tx) * at(ix, iy + 1) + tx * at(ix + 1, iy + 1));
}

unsigned grid1d(int64_t total, int64_t cap = 16384) {
  int64_t b = (total + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min(b, cap));
}

// ---------------------------------------------------------------- host side
struct Layout {
  int64_t oW1, ob1, oW2, ob2, oW3, ob3, total;  // FP32 flat offsets
  int64_t bW2, bW3, nb;                         // BF16 offsets
};
Layout layout_of(const klecgc_mlp* h) {
  Layout L;
  const int64_t H = h->hidden, O = h->n_out;
  L.oW1 = 0;
  L.ob1 = (int64_t)h->n_in * H;
  L.oW2 = L.ob1 + H;
  L.ob2 = L.oW2 + H * H;
  L.oW3 = L.ob2 + H;
  L.ob3 = L.oW3 + H * O;
  L.total = L.ob3 + O;
  L.bW2 = (int64_t)h->in_pad * H;
  L.bW3 = L.bW2 + H * H;
  L.nb = L.bW3 + H * O;
  return L;
}

constexpr int kSplitK = 32;      // partial sums for the K = n_out product
constexpr int kMseBlocksX = 64;  // column blocks of the loss-gradient kernel

struct Work {
  kc_bf16 *Xb, *h1b, *h2b, *dYb, *dp2b, *dp1b;
  float *pre1, *pre2, *Y, *dY, *dH2, *dp2, *dH1, *dp1, *part;
  double* loss;
  double* lpart;   // per-block loss partial sums [kMseBlocksX * B]
};

template <class T>
T* carve(char*& p, int64_t count) {
  T* r = reinterpret_cast<T*>(p);
  p += ((size_t)count * sizeof(T) + 255) & ~(size_t)255;
  return r;
}

size_t work_bytes(const klecgc_mlp* h, int B) {
  const int64_t H = h->hidden, O = h->n_out, P = h->in_pad;
  const int64_t nb = (int64_t)B * (P + 2 * H + O + 2 * H);
  const int64_t nf = (int64_t)B * (2 * H + 2 * O + 4 * H) + (int64_t)kSplitK * B * H;
  return (size_t)nb * 2 + (size_t)nf * 4 + (size_t)8 * kMseBlocksX * B + 18 * 256;
}

Work work_for(klecgc_ctx* ctx, klecgc_mlp* h, int B) {
  if (B > h->cap_b) {
    const size_t bytes = work_bytes(h, B);
    if (h->ws) {
      KC_TRY_HIP(hipStreamSynchronize(ctx->stream));
      KC_TRY_HIP(hipFree(h->ws));
      h->ws = nullptr;
      h->cap_b = 0;
    }
    if (hipMalloc(&h->ws, bytes) != hipSuccess) {
      (void)hipGetLastError();
      h->ws = nullptr;
      throw Error{KC_ENOMEM, "MLP work buffer allocation failed"};
    }
    h->ws_bytes = bytes;
    h->cap_b = B;
  }
  const int64_t H = h->hidden, O = h->n_out, P = h->in_pad;
  char* p = (char*)h->ws;
  Work w;
  w.Xb = carve<kc_bf16>(p, (int64_t)B * P);
  w.h1b = carve<kc_bf16>(p, (int64_t)B * H);
  w.h2b = carve<kc_bf16>(p, (int64_t)B * H);
  w.dYb = carve<kc_bf16>(p, (int64_t)B * O);
  w.dp2b = carve<kc_bf16>(p, (int64_t)B * H);
  w.dp1b = carve<kc_bf16>(p, (int64_t)B * H);
  w.pre1 = carve<float>(p, (int64_t)B * H);
  w.pre2 = carve<float>(p, (int64_t)B * H);
  w.Y = carve<float>(p, (int64_t)B * O);
  w.dY = carve<float>(p, (int64_t)B * O);
  w.dH2 = carve<float>(p, (int64_t)B * H);
  w.dp2 = carve<float>(p, (int64_t)B * H);
  w.dH1 = carve<float>(p, (int64_t)B * H);
  w.dp1 = carve<float>(p, (int64_t)B * H);
  w.part = carve<float>(p, (int64_t)kSplitK * B * H);
  w.loss = carve<double>(p, 1);
  w.lpart = carve<double>(p, (int64_t)kMseBlocksX * B);
  if ((size_t)(p - (char*)h->ws) > h->ws_bytes) throw Error{KC_EINVAL, "MLP work buffer layout overflow"};
  return w;
}

template <bool TA, bool TB, int EPI>
void gemm(hipStream_t s, int M, int N, int K, const kc_bf16* A, int lda, const kc_bf16* B, int ldb, float* C, int ldc,
          const float* bias = nullptr, kc_bf16* Cb = nullptr, int ldcb = 0) {
  const dim3 grid((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), 1);
  gemm_bf16_kernel<TA, TB, EPI><<<grid, dim3(256), 0, s>>>(M, N, K, K, A, lda, B, ldb, C, ldc, bias, Cb, ldcb);
  KC_LAUNCH_CHECK();
}

// C [M][N] (ldc = N) = A B^T over a long K: at most kSplitK partials in `part`, summed
void gemm_nt_splitk(hipStream_t s, int M, int N, int K, const kc_bf16* A, int lda, const kc_bf16* B, int ldb,
                    float* part, float* C) {
  int kchunk = (K + kSplitK - 1) / kSplitK;
  kchunk = (kchunk + GBK - 1) / GBK * GBK;
  const int S = (K + kchunk - 1) / kchunk;
  const dim3 grid((unsigned)((N + GBN - 1) / GBN), (unsigned)((M + GBM - 1) / GBM), (unsigned)S);
  gemm_bf16_kernel<false, true, EPI_STORE><<<grid, dim3(256), 0, s>>>(M, N, K, kchunk, A, lda, B, ldb, part, N,
                                                                      nullptr, nullptr, 0);
  KC_LAUNCH_CHECK();
  splitk_reduce_kernel<<<grid1d((int64_t)M * N), 256, 0, s>>>(part, S, (int64_t)M * N, C);
  KC_LAUNCH_CHECK();
}

void refresh_bf16(hipStream_t s, klecgc_mlp* h) {
  const Layout L = layout_of(h);
  const int64_t H = h->hidden;
  // W1 rows 0..n_in-1 keep their flat index; the padding rows stay zero
  KC_TRY_HIP(hipMemsetAsync(h->wb, 0, sizeof(kc_bf16) * L.bW2, s));
  to_bf16_kernel<<<grid1d(L.ob1), 256, 0, s>>>(h->w + L.oW1, L.ob1, h->wb);
  KC_LAUNCH_CHECK();
  to_bf16_kernel<<<grid1d(H * H), 256, 0, s>>>(h->w + L.oW2, H * H, h->wb + L.bW2);
  KC_LAUNCH_CHECK();
  to_bf16_kernel<<<grid1d(H * h->n_out), 256, 0, s>>>(h->w + L.oW3, H * h->n_out, h->wb + L.bW3);
  KC_LAUNCH_CHECK();
}

// forward of the B rows staged in w.Xb; the output goes to Yout [B][O]
void forward(hipStream_t s, const klecgc_mlp* h, const Work& w, int B, float* Yout) {
  const Layout L = layout_of(h);
  const int H = h->hidden, O = (int)h->n_out;
  gemm<false, false, EPI_BIAS_GELU>(s, B, H, h->in_pad, w.Xb, h->in_pad, h->wb, H, w.pre1, H, h->w + L.ob1, w.h1b, H);
  gemm<false, false, EPI_BIAS_GELU>(s, B, H, H, w.h1b, H, h->wb + L.bW2, H, w.pre2, H, h->w + L.ob2, w.h2b, H);
  gemm<false, false, EPI_BIAS>(s, B, O, H, w.h2b, H, h->wb + L.bW3, O, Yout, O, h->w + L.ob3);
}

// gradient of the batch loss into h->g; adds the batch sum of squared errors to w.loss
void backward(hipStream_t s, klecgc_mlp* h, const Work& w, int B, const float* Tg, const int32_t* perm,
              const TrainCtr* ctr, int64_t n_rows, int64_t off) {
  const Layout L = layout_of(h);
  const int H = h->hidden, O = (int)h->n_out;
  const float scale = (float)(2.0 / ((double)B * O));
  const unsigned gx = (unsigned)std::min<int64_t>((O + 255) / 256, kMseBlocksX);
  mse_grad_kernel<<<dim3(gx, (unsigned)B), 256, 0, s>>>(w.Y, Tg, perm, ctr, n_rows, off, O, scale, w.dY, w.dYb,
                                                       w.lpart);
  KC_LAUNCH_CHECK();
  loss_reduce_kernel<<<1, 256, 0, s>>>(w.lpart, (int64_t)gx * B, w.loss);
  KC_LAUNCH_CHECK();
  // layer 3: dW3 = h2b^T dYb, db3 = column sums of dY, dH2 = dYb W3b^T
  gemm<true, false, EPI_STORE>(s, H, O, B, w.h2b, H, w.dYb, O, h->g + L.oW3, O);
  colsum_kernel<<<(unsigned)((O + 63) / 64), 1024, 0, s>>>(w.dY, B, O, h->g + L.ob3);
  KC_LAUNCH_CHECK();
  gemm_nt_splitk(s, B, H, O, w.dYb, O, h->wb + L.bW3, O, w.part, w.dH2);
  gelu_bwd_kernel<<<grid1d((int64_t)B * H), 256, 0, s>>>(w.dH2, w.pre2, (int64_t)B * H, w.dp2, w.dp2b);
  KC_LAUNCH_CHECK();
  // layer 2
  gemm<true, false, EPI_STORE>(s, H, H, B, w.h1b, H, w.dp2b, H, h->g + L.oW2, H);
  colsum_kernel<<<(unsigned)((H + 63) / 64), 1024, 0, s>>>(w.dp2, B, H, h->g + L.ob2);
  KC_LAUNCH_CHECK();
  gemm<false, true, EPI_STORE>(s, B, H, H, w.dp2b, H, h->wb + L.bW2, H, w.dH1, H);
  gelu_bwd_kernel<<<grid1d((int64_t)B * H), 256, 0, s>>>(w.dH1, w.pre1, (int64_t)B * H, w.dp1, w.dp1b);
  KC_LAUNCH_CHECK();
  // layer 1 (the n_in real rows of W1)
  gemm<true, false, EPI_STORE>(s, h->n_in, H, B, w.Xb, h->in_pad, w.dp1b, H, h->g + L.oW1, H);
  colsum_kernel<<<(unsigned)((H + 63) / 64), 1024, 0, s>>>(w.dp1, B, H, h->g + L.ob1);
  KC_LAUNCH_CHECK();
}

void stage_x(hipStream_t s, const klecgc_mlp* h, const Work& w, const double* xi, const int32_t* perm,
             const TrainCtr* ctr, int64_t n_rows, int64_t off, int B) {
  gather_x_kernel<<<grid1d((int64_t)B * h->in_pad, 1 << 20), 256, 0, s>>>(xi, perm, ctr, n_rows, off, B, h->n_in,
                                                                          h->in_pad, w.Xb);
  KC_LAUNCH_CHECK();
}

}  // namespace

int64_t mlp_param_count(const klecgc_mlp* h) { return h->n_params; }
int64_t mlp_out_count(const klecgc_mlp* h) { return h->n_out; }
int mlp_in_count(const klecgc_mlp* h) { return h->n_in; }

int mlp_create_impl(klecgc_ctx* ctx, int n_in, int hidden, int64_t n_out, klecgc_mlp** out) {
  KC_REQUIRE(n_in >= 1 && n_in <= 4096, KC_EINVAL, "n_in must be in [1, 4096]");
  KC_REQUIRE(hidden >= 1 && hidden <= 16384, KC_EINVAL, "hidden must be in [1, 16384]");
  KC_REQUIRE(n_out >= 1 && n_out <= ((int64_t)1 << 30), KC_EINVAL, "n_out must be in [1, 2^30]");
  KC_REQUIRE((int64_t)hidden * n_out < ((int64_t)1 << 31), KC_EINVAL, "hidden * n_out must be < 2^31");
  auto* h = new klecgc_mlp;
  h->n_in = n_in;
  h->in_pad = (n_in + 15) / 16 * 16;
  h->hidden = hidden;
  h->n_out = n_out;
  const Layout L = layout_of(h);
  h->n_params = L.total;
  auto alloc = [&](void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      klecgc_mlp_free(h);
      throw Error{KC_ENOMEM, "MLP parameter allocation failed"};
    }
  };
  alloc((void**)&h->w, sizeof(float) * L.total);
  alloc((void**)&h->m, sizeof(float) * L.total);
  alloc((void**)&h->v, sizeof(float) * L.total);
  alloc((void**)&h->g, sizeof(float) * L.total);
  alloc((void**)&h->wb, sizeof(kc_bf16) * L.nb);
  alloc((void**)&h->mean, sizeof(float) * n_out);
  alloc((void**)&h->stdv, sizeof(float) * n_out);
  hipStream_t s = ctx->stream;
  try {
    KC_TRY_HIP(hipMemsetAsync(h->w, 0, sizeof(float) * L.total, s));
    KC_TRY_HIP(hipMemsetAsync(h->m, 0, sizeof(float) * L.total, s));
    KC_TRY_HIP(hipMemsetAsync(h->v, 0, sizeof(float) * L.total, s));
    KC_TRY_HIP(hipMemsetAsync(h->g, 0, sizeof(float) * L.total, s));
    KC_TRY_HIP(hipMemsetAsync(h->wb, 0, sizeof(kc_bf16) * L.nb, s));
    KC_TRY_HIP(hipMemsetAsync(h->mean, 0, sizeof(float) * n_out, s));
    fill_kernel<<<grid1d(n_out), 256, 0, s>>>(h->stdv, n_out, 1.0f);
    KC_LAUNCH_CHECK();
    KC_TRY_HIP(hipStreamSynchronize(s));
  } catch (...) {
    klecgc_mlp_free(h);
    throw;
  }
  *out = h;
  return KC_OK;
}

int mlp_set_params_impl(klecgc_ctx* ctx, klecgc_mlp* h, const float* params) {
  hipStream_t s = ctx->stream;
  KC_TRY_HIP(hipMemcpyAsync(h->w, params, sizeof(float) * h->n_params, hipMemcpyDeviceToDevice, s));
  KC_TRY_HIP(hipMemsetAsync(h->m, 0, sizeof(float) * h->n_params, s));
  KC_TRY_HIP(hipMemsetAsync(h->v, 0, sizeof(float) * h->n_params, s));
  h->t = 0;
  refresh_bf16(s, h);
  KC_TRY_HIP(hipStreamSynchronize(s));
  return KC_OK;
}

int mlp_get_params_impl(klecgc_ctx* ctx, const klecgc_mlp* h, float* params, float* mean, float* stdv) {
  hipStream_t s = ctx->stream;
  if (params) KC_TRY_HIP(hipMemcpyAsync(params, h->w, sizeof(float) * h->n_params, hipMemcpyDeviceToDevice, s));
  if (mean) KC_TRY_HIP(hipMemcpyAsync(mean, h->mean, sizeof(float) * h->n_out, hipMemcpyDeviceToDevice, s));
  if (stdv) KC_TRY_HIP(hipMemcpyAsync(stdv, h->stdv, sizeof(float) * h->n_out, hipMemcpyDeviceToDevice, s));
  return KC_OK;
}

int mlp_normalize_impl(klecgc_ctx* ctx, klecgc_mlp* h, float* Y, int64_t n) {
  zscore_kernel<<<grid1d(h->n_out, 1 << 20), 256, 0, ctx->stream>>>(Y, n, h->n_out, h->mean, h->stdv);
  KC_LAUNCH_CHECK();
  return KC_OK;
}

int mlp_predict_impl(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi, int64_t M, float* Y) {
  hipStream_t s = ctx->stream;
  const int chunk = 512;
  for (int64_t off = 0; off < M; off += chunk) {
    const int B = (int)std::min<int64_t>(chunk, M - off);
    Work w = work_for(ctx, h, B);
    stage_x(s, h, w, xi, nullptr, nullptr, M, off, B);
    timed(ctx, KT_MLP, [&] { forward(s, h, w, B, Y + off * h->n_out); });
  }
  return KC_OK;
}

int mlp_grad_impl(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi, const float* Y, int64_t n, float* grads,
                  double* loss) {
  hipStream_t s = ctx->stream;
  KC_REQUIRE(n >= 1 && n <= 65535, KC_EINVAL, "mlp_grad: n must be in [1, 65535]");
  Work w = work_for(ctx, h, (int)n);
  KC_TRY_HIP(hipMemsetAsync(w.loss, 0, sizeof(double), s));
  stage_x(s, h, w, xi, nullptr, nullptr, n, 0, (int)n);
  timed(ctx, KT_MLP, [&] {
    forward(s, h, w, (int)n, w.Y);
    backward(s, h, w, (int)n, Y, nullptr, nullptr, n, 0);
  });
  if (grads) KC_TRY_HIP(hipMemcpyAsync(grads, h->g, sizeof(float) * h->n_params, hipMemcpyDeviceToDevice, s));
  double hl = 0;
  KC_TRY_HIP(hipMemcpyAsync(&hl, w.loss, sizeof(double), hipMemcpyDeviceToHost, s));
  KC_TRY_HIP(hipStreamSynchronize(s));
  if (loss) *loss = hl / ((double)n * h->n_out);
  return KC_OK;
}

int mlp_train_impl(klecgc_ctx* ctx, klecgc_mlp* h, const double* xi, const float* Y, int64_t n, int epochs, int batch,
                   float lr, float lr_final, const int32_t* perm, float* loss_host) {
  hipStream_t s = ctx->stream;
  KC_REQUIRE(batch >= 1 && batch <= 65535, KC_EINVAL, "batch must be in [1, 65535]");
  KC_REQUIRE(epochs >= 0, KC_EINVAL, "epochs must be >= 0");
  KC_REQUIRE(lr > 0.f && std::isfinite(lr), KC_EINVAL, "lr must be positive and finite");
  KC_REQUIRE(std::isfinite(lr_final), KC_EINVAL, "lr_final must be finite");
  const Layout L = layout_of(h);
  const AdamSeg sg{L.oW2, L.ob2, L.oW3, L.ob3, L.bW2, L.bW3};
  const int64_t nbatch = (n + batch - 1) / batch;
  Work w = work_for(ctx, h, (int)std::min<int64_t>(batch, n));
  KC_REQUIRE(n <= INT32_MAX, KC_EINVAL, "n must fit int32 row indices");
  if (perm && epochs > 0) {
    int* flag = (int*)ctx->ws.get(WS_SMALL, 256);
    KC_TRY_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    check_perm_kernel<<<grid1d((int64_t)epochs * n), 256, 0, s>>>(perm, (int64_t)epochs * n, (int32_t)n, flag);
    KC_LAUNCH_CHECK();
    int hf = 0;
    KC_TRY_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    KC_TRY_HIP(hipStreamSynchronize(s));
    KC_REQUIRE(hf == 0, KC_EINVAL, "perm_dev holds a row index outside [0, n)");
  }
  if (epochs == 0) return KC_OK;
  // One epoch of steps is captured into a graph on a library-owned stream (a caller's
  // legacy null stream cannot be captured) and replayed `epochs` times; the step count,
  // the epoch index and the loss accumulator live in device memory.
  struct Owned {
    void* buf = nullptr;
    hipStream_t cs = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~Owned() {
      if (cs) (void)hipStreamSynchronize(cs);
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      if (cs) (void)hipStreamDestroy(cs);
      if (buf) (void)hipFree(buf);
    }
  } o;
  KC_TRY_HIP(hipMalloc(&o.buf, 256 + sizeof(double) * (size_t)epochs));
  TrainCtr* ctr = (TrainCtr*)o.buf;
  double* hist = (double*)((char*)o.buf + 256);
  KC_TRY_HIP(hipStreamCreateWithFlags(&o.cs, hipStreamNonBlocking));
  KC_TRY_HIP(hipEventCreate(&o.e0));
  KC_TRY_HIP(hipEventCreate(&o.e1));
  const TrainCtr c0{h->t, 0};
  KC_TRY_HIP(hipMemcpyAsync(ctr, &c0, sizeof(c0), hipMemcpyHostToDevice, s));
  KC_TRY_HIP(hipMemsetAsync(w.loss, 0, sizeof(double), s));
  KC_TRY_HIP(hipEventRecord(o.e0, s));
  KC_TRY_HIP(hipStreamWaitEvent(o.cs, o.e0, 0));
  hipStream_t cs = o.cs;
  KC_TRY_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  try {
    for (int64_t bi = 0; bi < nbatch; ++bi) {
      const int64_t off = bi * batch;
      const int B = (int)std::min<int64_t>(batch, n - off);
      stage_x(cs, h, w, xi, perm, ctr, n, off, B);
      forward(cs, h, w, B, w.Y);
      backward(cs, h, w, B, Y, perm, ctr, n, off);
      adam_kernel<<<grid1d(h->n_params), 256, 0, cs>>>(h->w, h->g, h->m, h->v, h->n_params, lr, lr_final, epochs,
                                                       0.9f, 0.999f, 1e-8f, ctr, L.ob1, sg, h->wb);
      KC_LAUNCH_CHECK();
      step_kernel<<<1, 64, 0, cs>>>(ctr);
      KC_LAUNCH_CHECK();
    }
    epoch_end_kernel<<<1, 64, 0, cs>>>(ctr, w.loss, hist, 1.0 / ((double)n * h->n_out));
    KC_LAUNCH_CHECK();
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  KC_TRY_HIP(hipStreamEndCapture(cs, &o.g));
  KC_TRY_HIP(hipGraphInstantiate(&o.x, o.g, nullptr, nullptr, 0));
  KC_TRY_HIP(hipEventRecord(o.e0, cs));
  for (int ep = 0; ep < epochs; ++ep) KC_TRY_HIP(hipGraphLaunch(o.x, cs));
  KC_TRY_HIP(hipEventRecord(o.e1, cs));
  std::vector<double> hl((size_t)epochs);
  KC_TRY_HIP(hipMemcpyAsync(hl.data(), hist, sizeof(double) * epochs, hipMemcpyDeviceToHost, cs));
  KC_TRY_HIP(hipStreamSynchronize(cs));
  float ms = 0.f;
  KC_TRY_HIP(hipEventElapsedTime(&ms, o.e0, o.e1));
  ctx->ktime[KT_MLP] += ms;
  ctx->kcount[KT_MLP] += epochs;
  h->t += (int64_t)epochs * nbatch;
  if (loss_host)
    for (int ep = 0; ep < epochs; ++ep) loss_host[ep] = (float)hl[ep];
  // the caller's stream resumes after the training
  KC_TRY_HIP(hipEventRecord(o.e1, cs));
  KC_TRY_HIP(hipStreamWaitEvent(s, o.e1, 0));
  return KC_OK;
}

int grid_restrict_impl(klecgc_ctx* ctx, int n, int nc, const double* U, int64_t R, float* Yc) {
  for (int64_t r0 = 0; r0 < R; r0 += 65535) {
    const int64_t Rc = std::min<int64_t>(65535, R - r0);
    restrict_kernel<<<dim3((unsigned)((nc * nc + 255) / 256), (unsigned)Rc), 256, 0, ctx->stream>>>(
        U + r0 * (int64_t)n * n, n, nc, Rc, Yc + r0 * (int64_t)nc * nc);
    KC_LAUNCH_CHECK();
  }
  return KC_OK;
}

int mlp_initial_guess_impl(klecgc_ctx* ctx, klecgc_mlp* h, int n, int nc, int N, const double* xi, int64_t M,
                           double* U0) {
  KC_REQUIRE(h->n_out == (int64_t)N * nc * nc, KC_EINVAL, "MLP output size must equal N * nc^2");
  float* Yz = (float*)ctx->ws.get(WS_MLP, sizeof(float) * M * h->n_out);
  mlp_predict_impl(ctx, h, xi, M, Yz);
  const int64_t MN = M * N;
  for (int64_t r0 = 0; r0 < MN; r0 += 65535) {
    const int64_t Rc = std::min<int64_t>(65535, MN - r0);
    prolong_kernel<<<dim3((unsigned)(((int64_t)n * n + 255) / 256), (unsigned)Rc), 256, 0, ctx->stream>>>(
        Yz + r0 * (int64_t)nc * nc, h->mean, h->stdv, n, nc, N, r0, Rc, U0 + r0 * (int64_t)n * n);
    KC_LAUNCH_CHECK();
  }
  return KC_OK;
}

}  // namespace kc

extern "C" void klecgc_mlp_free(klecgc_mlp* h) {
  if (!h) return;
  (void)hipFree(h->w);
  (void)hipFree(h->m);
  (void)hipFree(h->v);
  (void)hipFree(h->g);
  (void)hipFree(h->wb);
  (void)hipFree(h->mean);
  (void)hipFree(h->stdv);
  (void)hipFree(h->ws);
  delete h;
}
