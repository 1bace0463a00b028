// Dense float64 GEMM on the CDNA matrix cores (v_mfma_f64_16x16x4f64), plus the small
// kernels of the KL / gPC stages (Section 2.1, Section 2.2, Algorithm 3):
//   * gPC tensor basis (Hermite or Legendre) Psi[m][i] = prod_l psi_{k_il}(xi_ml)
//   * column mean of the snapshot matrix and its centred copy
//   * C = bias + alpha * op(A) op(B) used for the Gram matrix S~ S~^T, the basis
//     E^T S~ and the prediction Psi H W.
#include "common.h"

namespace kc {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16;

// Work-group of 4 waves computes a 64x64 tile; wave w owns the 32x32 quadrant
// (w / 2, w % 2) as 2x2 MFMA 16x16 blocks.  MFMA f64 16x16x4 operand layout:
// A: lane l holds A[l % 16][l / 16]; B: lane l holds B[l / 16][l % 16];
// D: lane l, element e holds D[4 * e + l / 16][l % 16] (measured on gfx950).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void dgemm_kernel(int64_t Mr, int64_t Nc, int64_t K,
                                                    const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    double* __restrict__ C, int64_t ldc,
                                                    const double* __restrict__ bias, double alpha) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t row0 = (int64_t)blockIdx.y * BM;
  const int64_t col0 = (int64_t)blockIdx.x * BN;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  double4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};

  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    // stage A tile (BM x BK) as As[k][i] and B tile (BK x BN) as Bs[k][j]
#pragma unroll
    for (int e = 0; e < (BM * BK) / 256; ++e) {
      int idx = tid + e * 256;
      int i, k;
      if (TA) {        // A stored [K][M]: consecutive threads along i
        i = idx % BM;
        k = idx / BM;
      } else {         // A stored [M][K]: consecutive threads along k
        k = idx % BK;
        i = idx / BK;
      }
      int64_t gi = row0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < Mr && gk < K) v = TA ? A[gk * lda + gi] : A[gi * lda + gk];
      As[k][i] = v;
    }
#pragma unroll
    for (int e = 0; e < (BN * BK) / 256; ++e) {
      int idx = tid + e * 256;
      int j, k;
      if (TB) {        // B stored [N][K]
        k = idx % BK;
        j = idx / BK;
      } else {         // B stored [K][N]
        j = idx % BN;
        k = idx / BN;
      }
      int64_t gj = col0 + j, gk = k0 + k;
      double v = 0.0;
      if (gj < Nc && gk < K) v = TB ? B[gj * ldb + gk] : B[gk * ldb + gj];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) af[a] = As[kk + lane / 16][wr + a * 16 + lane % 16];
#pragma unroll
      for (int b = 0; b < 2; ++b) bf[b] = Bs[kk + lane / 16][wc + b * 16 + lane % 16];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t gi = row0 + wr + a * 16 + 4 * e + lane / 16;
        int64_t gj = col0 + wc + b * 16 + lane % 16;
        if (gi < Mr && gj < Nc) {
          double v = alpha * acc[a][b][e];
          if (bias) v += bias[gj];
          C[gi * ldc + gj] = v;
        }
      }
}

__global__ void gpc_basis_kernel(const double* __restrict__ xi, int64_t M, int d,
                                 const int32_t* __restrict__ idx, int P, int basis,
                                 double* __restrict__ Psi) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * P) return;
  int64_t m = t / P;
  int i = (int)(t % P);
  double prod = 1.0;
  for (int l = 0; l < d; ++l) {
    int k = idx[i * d + l];
    if (k == 0) continue;
    double x = xi[m * d + l];
    double pm1 = 1.0, pj = x;
    if (basis == KC_GPC_LEGENDRE) {
      // Bonnet: (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}; orthonormal under U(-1,1): sqrt(2k+1) P_k
      for (int j = 1; j < k; ++j) {
        double nx = ((2.0 * j + 1.0) * x * pj - (double)j * pm1) / (double)(j + 1);
        pm1 = pj;
        pj = nx;
      }
      pj *= sqrt(2.0 * k + 1.0);
    } else {
      // orthonormal probabilists' Hermite: psi_{j+1} = (x psi_j - sqrt(j) psi_{j-1}) / sqrt(j+1)
      for (int j = 1; j < k; ++j) {
        double nx = (x * pj - sqrt((double)j) * pm1) / sqrt((double)(j + 1));
        pm1 = pj;
        pj = nx;
      }
    }
    prod *= pj;
  }
  Psi[m * P + i] = prod;
}

// mean[c] = (1/n_t) sum_r S[r][c]; Sc = S - mean (row-wise)
__global__ void col_mean_center_kernel(const double* __restrict__ S, int64_t n_t, int64_t L,
                                       double* __restrict__ mean, double* __restrict__ Sc) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= L) return;
  double s = 0.0;
  for (int64_t r = 0; r < n_t; ++r) s += S[r * L + c];
  s /= (double)n_t;
  mean[c] = s;
  if (Sc)
    for (int64_t r = 0; r < n_t; ++r) Sc[r * L + c] = S[r * L + c] - s;
}

}  // namespace

void launch_dgemm(hipStream_t s, int64_t Mr, int64_t Nc, int64_t K, const double* A, int64_t lda,
                  const double* B, int64_t ldb, double* C, int64_t ldc, const double* bias,
                  double alpha) {
  dim3 grid((unsigned)((Nc + BN - 1) / BN), (unsigned)((Mr + BM - 1) / BM));
  dgemm_kernel<false, false><<<grid, dim3(256), 0, s>>>(Mr, Nc, K, A, lda, B, ldb, C, ldc, bias, alpha);
  KC_LAUNCH_CHECK();
}

// C[Mr][Nc] = alpha * A B^T with A [Mr][K], B [Nc][K]   (Gram matrices)
void launch_dgemm_nt(hipStream_t s, int64_t Mr, int64_t Nc, int64_t K, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                     double alpha) {
  dim3 grid((unsigned)((Nc + BN - 1) / BN), (unsigned)((Mr + BM - 1) / BM));
  dgemm_kernel<false, true><<<grid, dim3(256), 0, s>>>(Mr, Nc, K, A, lda, B, ldb, C, ldc, nullptr, alpha);
  KC_LAUNCH_CHECK();
}

// C[Mr][Nc] = alpha * A^T B with A [K][Mr], B [K][Nc]
void launch_dgemm_tn(hipStream_t s, int64_t Mr, int64_t Nc, int64_t K, const double* A,
                     int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                     double alpha) {
  dim3 grid((unsigned)((Nc + BN - 1) / BN), (unsigned)((Mr + BM - 1) / BM));
  dgemm_kernel<true, false><<<grid, dim3(256), 0, s>>>(Mr, Nc, K, A, lda, B, ldb, C, ldc, nullptr, alpha);
  KC_LAUNCH_CHECK();
}

void launch_gpc_basis(hipStream_t s, const double* xi, int64_t M, int d, const int32_t* idx, int P,
                      int basis, double* Psi) {
  int64_t tot = M * P;
  gpc_basis_kernel<<<dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s>>>(xi, M, d, idx, P, basis, Psi);
  KC_LAUNCH_CHECK();
}

void launch_col_mean_center(hipStream_t s, const double* S, int64_t n_t, int64_t L, double* mean,
                            double* Sc) {
  col_mean_center_kernel<<<dim3((unsigned)((L + 255) / 256)), dim3(256), 0, s>>>(S, n_t, L, mean, Sc);
  KC_LAUNCH_CHECK();
}

}  // namespace kc
