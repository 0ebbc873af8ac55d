// The lower part of the V-cycle (Alg. 7) as one dense operator.
//
// Below the finest level, one V-cycle from a zero start with damped Jacobi
// smoothing (Alg. 6) and the direct coarse solve (Sec. 3.2.4) is a fixed
// linear map of its right-hand side, alpha = B_g b. Written for every column
// of the identity at once, the steps of Alg. 7 give B_g from B_{g-1}:
//   M1  = sum_{j < nu1} (I - W A)^j W          (nu1 sweeps from zero)
//   X   = M1 + I_g (B_{g-1} (I_g' (I - A M1)))   (coarse-grid correction)
//   B_g = X + W (I - A X), nu2 times            (post-smoothing)
// with A = A_g assembled from its stencil, W = omega_g D_g^-1 and I_g the
// subdivision matrix of eq. 2.5. Each step is a product of dense matrices:
// the GEMMs below run on the FP64 matrix cores. The V-cycle from that level
// down then takes one matrix-vector product instead of two stencil products,
// two transfers and the coarse solve per level, each a launch of a few
// microseconds on levels this small.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace tsmg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;      // block tile (rows and columns of C)
constexpr int kGK = 16;      // k step staged in LDS
constexpr int kGThreads = 256;

// C = base + rs .* (dlt I + sgn A B), A: M x Kd, B: Kd x N, all row-major
// FP64 (base, rs may be null; C must not alias A or B; base may alias C).
// Four wavefronts per 64 x 64 tile, each a 32 x 32 quarter as 2 x 2 tiles
// of the 16 x 16 x 4 FP64 matrix instruction: lane l supplies A[l % 16][k0 +
// l / 16] and B[k0 + l / 16][l % 16] and holds D[4 r + l / 16][l % 16] in its
// result register r = 0..3. Tiles past the edges are read as zeros.
__global__ __launch_bounds__(kGThreads) void k_gemm64(const double* __restrict__ A, const double* __restrict__ B,
                                                      int M, int N, int Kd, const double* base,
                                                      const double* __restrict__ rs, double dlt, double sgn,
                                                      double* C) {
  __shared__ double As[kGK][kGT + 1];   // [k][row]
  __shared__ double Bs[kGK][kGT + 1];   // [k][col]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int bm = blockIdx.y * kGT, bn = blockIdx.x * kGT;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < Kd; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < kGT * kGK / kGThreads; ++i) {
      const int e = tid + kGThreads * i;
      const int r = e >> 4, kk = e & 15;   // A: 16 consecutive k of one row
      const int gr = bm + r, gk = k0 + kk;
      As[kk][r] = (gr < M && gk < Kd) ? A[size_t(gr) * Kd + gk] : 0.0;
      const int kb = e >> 6, c = e & 63;   // B: 64 consecutive columns of one k
      const int gkb = k0 + kb, gc = bn + c;
      Bs[kb][c] = (gkb < Kd && gc < N) ? B[size_t(gkb) * N + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 4) {
      const int kk = ks + lk;
      const double a0 = As[kk][wm + li], a1 = As[kk][wm + 16 + li];
      const double b0 = Bs[kk][wn + li], b1 = Bs[kk][wn + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = bm + wm + a * 16 + 4 * r + lk;
        const int col = bn + wn + b * 16 + li;
        if (row < M && col < N) {
          double v = sgn * acc[a][b][r] + (row == col ? dlt : 0.0);
          if (rs) v *= rs[row];
          const size_t o = size_t(row) * N + col;
          if (base) v += base[o];
          C[o] = v;
        }
      }
}

// Dense subdivision matrix of one level pair: R[j][i] = prod_p r(j_p, i_p)
// with the 1D restriction weights r(j, i) = binom(4, i - 2 j + 3) / 8 (the
// transpose of eq. 2.5), C-order indices over Jc^D coarse and Jf^D fine
// coefficients; with transpose set, the prolongation P = R' (Jf^D x Jc^D).
__global__ __launch_bounds__(kBlock) void k_subdivision_dense(double* out, int D, int Jc, int Jf, int64_t Kc,
                                                              int64_t Kf, int transpose) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= Kc * Kf) return;
  int64_t j = transpose ? t % Kc : t / Kf;
  int64_t i = transpose ? t / Kc : t % Kf;
  const double b4[5] = {0.125, 0.5, 0.75, 0.5, 0.125};
  double v = 1.0;
  for (int p = 0; p < D && v != 0.0; ++p) {
    const int jp = int(j % Jc), ip = int(i % Jf);
    j /= Jc;
    i /= Jf;
    const int m = ip - 2 * jp + 3;
    v *= (m >= 0 && m <= 4) ? b4[m] : 0.0;
  }
  out[t] = v;
}

// out = diag(w) (K x K).
__global__ __launch_bounds__(kBlock) void k_diag_dense(const double* w, int64_t K, double* out) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= K * K) return;
  const int64_t r = t / K, c = t % K;
  out[t] = (r == c) ? w[r] : 0.0;
}

// out = I - A diag(w) (K x K): the residual map after one sweep from zero.
__global__ __launch_bounds__(kBlock) void k_eye_minus_scaled(const double* A, const double* w, int64_t K,
                                                             double* out) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= K * K) return;
  const int64_t r = t / K, c = t % K;
  out[t] = (r == c ? 1.0 : 0.0) - A[t] * w[c];
}

// s_i = 1 / sqrt(A_ii) (NaN where A_ii <= 0, which the pivot test then rejects).
__global__ __launch_bounds__(kBlock) void k_inv_sqrt_diag(const double* A, int K, double* s) {
  const int i = int(blockIdx.x) * kBlock + threadIdx.x;
  if (i < K) s[i] = 1.0 / sqrt(A[size_t(i) * K + i]);
}

// A_ij *= s_i s_j (K x K, in place).
__global__ __launch_bounds__(kBlock) void k_sym_scale(double* A, int K, const double* s) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= int64_t(K) * K) return;
  A[t] *= s[t / K] * s[t % K];
}

// out (cols x rows) = in' (in: rows x cols).
__global__ __launch_bounds__(kBlock) void k_transpose(const double* in, int64_t rows, int64_t cols, double* out) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= rows * cols) return;
  const int64_t r = t / cols, c = t % cols;
  out[c * rows + r] = in[t];
}

__global__ __launch_bounds__(kBlock) void k_round_f32(const double* in, int64_t n, float* out) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t < n) out[t] = float(in[t]);
}

// out = B v for the dense K x K operator B, one wavefront per row with four
// independent partial sums, FP64 accumulation.
template <typename TM, typename TV>
__global__ __launch_bounds__(kBlock) void k_bottom_gemv(const TM* __restrict__ B, int K, const TV* __restrict__ v,
                                                        TV* __restrict__ out) {
  const int row = int((int64_t(blockIdx.x) * kBlock + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= K) return;
  const TM* br = B + size_t(row) * K;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = lane;
  for (; j + 192 < K; j += 256) {
    s0 += double(br[j]) * double(v[j]);
    s1 += double(br[j + 64]) * double(v[j + 64]);
    s2 += double(br[j + 128]) * double(v[j + 128]);
    s3 += double(br[j + 192]) * double(v[j + 192]);
  }
  for (; j < K; j += 64) s0 += double(br[j]) * double(v[j]);
  double acc = (s0 + s1) + (s2 + s3);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) out[row] = TV(acc);
}

unsigned blocks_of(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_gemm64(const double* A, const double* B, int M, int N, int Kd, const double* base,
                         const double* rs, double dlt, double sgn, double* C, hipStream_t st) {
  if (M <= 0 || N <= 0 || Kd <= 0) return hipErrorInvalidValue;
  const dim3 grid(unsigned((N + kGT - 1) / kGT), unsigned((M + kGT - 1) / kGT));
  hipLaunchKernelGGL(k_gemm64, grid, dim3(kGThreads), 0, st, A, B, M, N, Kd, base, rs, dlt, sgn, C);
  return hipGetLastError();
}

hipError_t launch_subdivision_dense(double* out, int D, int Jc, int Jf, bool transpose, hipStream_t st) {
  int64_t Kc = 1, Kf = 1;
  for (int p = 0; p < D; ++p) { Kc *= Jc; Kf *= Jf; }
  hipLaunchKernelGGL(k_subdivision_dense, dim3(blocks_of(Kc * Kf)), dim3(kBlock), 0, st, out, D, Jc, Jf, Kc, Kf,
                     transpose ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_diag_dense(const double* w, int64_t K, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_dense, dim3(blocks_of(K * K)), dim3(kBlock), 0, st, w, K, out);
  return hipGetLastError();
}

hipError_t launch_eye_minus_scaled(const double* A, const double* w, int64_t K, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_eye_minus_scaled, dim3(blocks_of(K * K)), dim3(kBlock), 0, st, A, w, K, out);
  return hipGetLastError();
}

hipError_t launch_inv_sqrt_diag(const double* A, int K, double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_inv_sqrt_diag, dim3(blocks_of(K)), dim3(kBlock), 0, st, A, K, s);
  return hipGetLastError();
}

hipError_t launch_sym_scale(double* A, int K, const double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_sym_scale, dim3(blocks_of(int64_t(K) * K)), dim3(kBlock), 0, st, A, K, s);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* in, int64_t rows, int64_t cols, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_transpose, dim3(blocks_of(rows * cols)), dim3(kBlock), 0, st, in, rows, cols, out);
  return hipGetLastError();
}

hipError_t launch_round_f32(const double* in, int64_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_round_f32, dim3(blocks_of(n)), dim3(kBlock), 0, st, in, n, out);
  return hipGetLastError();
}

template <typename TM, typename TV>
hipError_t launch_bottom_gemv(const TM* B, int K, const TV* v, TV* out, hipStream_t st) {
  hipLaunchKernelGGL((k_bottom_gemv<TM, TV>), dim3(blocks_of(int64_t(K) * 64)), dim3(kBlock), 0, st, B, K, v, out);
  return hipGetLastError();
}
template hipError_t launch_bottom_gemv<double, double>(const double*, int, const double*, double*, hipStream_t);
template hipError_t launch_bottom_gemv<float, float>(const float*, int, const float*, float*, hipStream_t);

}  // namespace tsmg
