// Host-side launchers of the tsmg kernels (defined in kernels.hip).
#pragma once
#include "common.h"

namespace tsmg {

constexpr int kMaxPartials = 1024;   // partial sums per reduction

struct BoxArgs {
  double lo[kMaxDim];
  double hi[kMaxDim];
  double inv_h[kMaxDim];   // N / (hi - lo)
  int G;                   // N = 2^G intervals per dimension
};

template <typename T>
struct LambdaArgs {
  const T* in0; const T* in1; const T* in2;   // T0, T1, T2 (in1/in2 unused when first)
  T* out0; T* out1; T* out2;                  // next T0, T1, T2 (unused when last)
  T* out;                                     // lambda * T2 (last pass only)
  const T* band;                              // [3][J][7]: M, G1, G2
  int64_t K;                                  // J^D
  int64_t stride;                             // J^(D-1-p)
  int J;
  int first, last;
  T lam;
};

template <typename T>
struct TransferArgs {
  const T* in;
  T* out;
  int64_t Kout;     // output length
  int64_t inner;    // product of the sizes of the dimensions after p
  int Jc, Jf;       // coarse / fine length of dimension p
  int subtract;     // prolongation only: out -= value instead of out = value
  const T* sub;     // restriction only: input is in - sub (null: in)
  const T* w;       // restriction only, with a: also a = w .* out (the coarse
  T* a;             // level's first Jacobi sweep from zero); a null: not done
};

hipError_t launch_data(int D, bool fp32, int mode, const DataArgs& a, hipStream_t st);

template <typename T> hipError_t launch_lambda_pass(const LambdaArgs<T>& a, hipStream_t st);
// out = lam * Lambda c in one kernel (d = 2 or 3); band: d blocks of [3][J][7].
template <typename T>
hipError_t launch_lambda_fused(int D, const T* c, T* out, const T* band, int J, T lam, hipStream_t st);
// out = lam * (the last three dimensions of the recursion) applied to
// (t0, t1, t2) for each of `outer` leading blocks of J^3 entries; band: the
// factors of those three dimensions, [3][3][J][7].
template <typename T>
hipError_t launch_lambda_tail3(const T* t0, const T* t1, const T* t2, T* out, const T* band, int J, int64_t outer,
                               T lam, hipStream_t st);
hipError_t launch_lambda_diag(int D, const double* band, int J, int64_t K, double lam, double* out,
                              hipStream_t st);
template <typename T> hipError_t launch_transfer(bool prolong, const TransferArgs<T>& a, hipStream_t st);
// Whole transfer in one kernel (small levels): prolongation out (=|-=) I in,
// or restriction out = I'(in - sub) (sub may be null), which with aj non-null
// also writes aj = wj .* out (the coarse level's first Jacobi sweep from zero).
template <typename T>
hipError_t launch_transfer_fused(int D, bool prolong, const T* in, const T* sub, T* out, int Jc, int Jf,
                                 int subtract, const T* wj, T* aj, hipStream_t st);
constexpr int64_t kFusedTransferMaxK = 65536;   // fine-level size up to which the fused form is used

template <typename T> hipError_t launch_jacobi_first(T* alpha, const T* wdinv, const T* b, int64_t K, hipStream_t st);
template <typename T> hipError_t launch_jacobi(T* alpha, const T* wdinv, const T* b, const T* Ax, int64_t K,
                                               hipStream_t st);
template <typename T> hipError_t launch_residual(T* r, const T* Ax, const T* b, int64_t K, hipStream_t st);

template <typename TX, typename TY>
hipError_t launch_dot(const TX* x, const TY* y, int64_t K, double* partial, double* slot, hipStream_t st);
template <typename TA, typename T>
hipError_t launch_cg_step(TA* alpha, T* r, const T* p, const T* v, int64_t K, const double* num,
                          const double* den, hipStream_t st);
// FP64 CG step fused with *rr = r'r and (z non-null) *rz = r'z of the
// updated r, and (zf non-null) zf = wz .* r; partial holds 2 * kMaxPartials.
// With den_part non-null the step's denominator is the sum of those den_nb
// partials (the first stage of p'v), also stored to *den.
hipError_t launch_cg_step_norms(double* alpha, double* r, const double* p, const double* v, const double* z,
                                int64_t K, const double* num, double* den, double* partial, double* rr,
                                double* rz, const double* wz, double* zf, const double* den_part, int den_nb,
                                hipStream_t st);
// The first stage of x'y alone: per-block partials (*nb of them).
template <typename TX, typename TY>
hipError_t launch_dot_partial(const TX* x, const TY* y, int64_t K, double* partial, int* nb, hipStream_t st);
// FP64 p = z + beta p, beta = (sum of the nb partials num_part - *sub) / *den
// (sub may be null); the sum is stored to *num.
hipError_t launch_p_update_sum(double* p, const double* z, int64_t K, double* num, const double* num_part, int nb,
                               const double* sub, const double* den, hipStream_t st);
template <typename T>
hipError_t launch_p_update(T* p, const T* z, int64_t K, const double* num, const double* den, hipStream_t st);
template <typename TI, typename TO>
hipError_t launch_scale_copy(const TI* x, TO* y, int64_t K, double scale, const double* sden, hipStream_t st);
// y = sqrt(*smul) x
hipError_t launch_scale_mul(const float* x, double* y, int64_t K, const double* smul, hipStream_t st);
template <typename TI, typename TO>
hipError_t launch_axpy_conv(const TI* x, TO* y, int64_t K, double scale, const double* smul, hipStream_t st);

hipError_t launch_mul(const double* d, const double* x, double* y, int64_t K, hipStream_t st);
// w = d .* Ax - sqrt(*b2prev) vprev (b2prev NULL: no vprev term)
hipError_t launch_lanczos_w(const double* d, const double* Ax, const double* vprev, const double* b2prev, double* w,
                            int64_t K, hipStream_t st);
// y += (scale * *s) x, s on the device
hipError_t launch_axpy(double scale, const double* s, const double* x, double* y, int64_t K, hipStream_t st);
hipError_t launch_start_vector(double* u, int64_t K, hipStream_t st);
hipError_t launch_rsqrt_vec(const double* D, double* out, int64_t K, hipStream_t st);
hipError_t launch_wdinv(const double* D, double omega, double* w64, float* w32, int64_t K, hipStream_t st);
template <typename T> hipError_t launch_fill(T* x, T v, int64_t K, hipStream_t st);
hipError_t launch_check_finite(const double* x, int64_t K, int* flag, hipStream_t st);

hipError_t launch_bin(int D, const double* x, int64_t n, const BoxArgs& box, uint32_t* key, uint32_t* idx,
                      int* flag, hipStream_t st);
hipError_t launch_place(int D, const double* x, const double* y, const uint32_t* idx, int64_t n,
                        const BoxArgs& box, double* t64, float* t32, uint32_t* cell, double* ys, hipStream_t st);
hipError_t launch_offsets(const uint32_t* key, int64_t n, int64_t ncells, int32_t* off, hipStream_t st);
hipError_t launch_eval(int D, const double* alpha, const double* xq, int64_t m, const BoxArgs& box, double* yq,
                       hipStream_t st);

hipError_t launch_dense_from_stencil(int D, const double* S, int J, int64_t K, double* A, hipStream_t st);
hipError_t launch_gj_step(double* A, int K, int k, double* row, double* col, double* piv, hipStream_t st);
hipError_t launch_symmetrize(double* A, int K, hipStream_t st);
// out = base + s * A v (dense K x K, FP64 arithmetic); base may be null.
template <typename TB, typename TV, typename TO>
hipError_t launch_gemv(const double* A, int K, const TB* base, double s, const TV* v, TO* out, hipStream_t st);

// Dense V-cycle operator of the lower levels (bottom.hip).
// C = base + rs .* (dlt I + sgn A B) for row-major FP64 A (M x Kd) and B
// (Kd x N) on the matrix cores; base and rs may be null, C must not alias A
// or B (base may alias C).
hipError_t launch_gemm64(const double* A, const double* B, int M, int N, int Kd, const double* base,
                         const double* rs, double dlt, double sgn, double* C, hipStream_t st);
// The dense subdivision restriction Jc^D x Jf^D (eq. 2.5 transposed), or with
// transpose set the prolongation Jf^D x Jc^D.
hipError_t launch_subdivision_dense(double* out, int D, int Jc, int Jf, bool transpose, hipStream_t st);
hipError_t launch_diag_dense(const double* w, int64_t K, double* out, hipStream_t st);
// out = I - A diag(w)
hipError_t launch_eye_minus_scaled(const double* A, const double* w, int64_t K, double* out, hipStream_t st);
hipError_t launch_round_f32(const double* in, int64_t n, float* out, hipStream_t st);
// out (cols x rows) = in' for a row-major rows x cols matrix
hipError_t launch_transpose(const double* in, int64_t rows, int64_t cols, double* out, hipStream_t st);
// s = diag(A)^-1/2 of a dense K x K matrix; A_ij *= s_i s_j
hipError_t launch_inv_sqrt_diag(const double* A, int K, double* s, hipStream_t st);
hipError_t launch_sym_scale(double* A, int K, const double* s, hipStream_t st);
// out = B v (dense K x K, FP64 accumulation)
template <typename TM, typename TV>
hipError_t launch_bottom_gemv(const TM* B, int K, const TV* v, TV* out, hipStream_t st);

// Assembled 7^D stencil of a level (moments -> D Kronecker passes -> finalize).
hipError_t launch_level_moments(int D, const double* t64, const uint32_t* cell, const int32_t* off, int64_t n,
                                int G, int g, double* mom, bool det, hipStream_t st);
// One dimension of the level g -> g-1 moment change of variables (Nc = N_{g-1}).
hipError_t launch_moments_coarsen(const double* in, double* out, int Nc, int64_t outer, int64_t inner,
                                  hipStream_t st);
hipError_t launch_stencil_pass(const double* in, double* out, const double* ctab, int N, int64_t outer,
                               int64_t inner, hipStream_t st);
hipError_t launch_stencil_finalize(int D, const double* inter, const double* band, int J, int64_t K, double lam,
                                   double* S64, float* S32, hipStream_t st);
// epi: 0 out = A x; 1 out = x + w (b - A x); 2 out = A x - b; 3 two Jacobi sweeps
// from zero, out = x1 + w (b - A x1) with x1 = w b (x unused). out must not
// alias x, b or w.
template <typename T>
hipError_t launch_stencil_apply(int D, int epi, const T* S, int J, const T* x, T* out, const T* b, const T* w,
                                int64_t K, hipStream_t st);

// One colour class of the SSOR sweep on a stencil level, in place:
// x_k += omega (b_k - (A x)_k) / A_kk for the rows with j_p = c_p (mod 4),
// c_p the base-4 digits of `color` (C order); 4^D classes.
template <typename T>
hipError_t launch_stencil_color(int D, const T* S, int J, T* x, const T* b, T omega, int color, int64_t K,
                                hipStream_t st);

// Radix sort of (key, index) pairs on the low `bits` bits (sort.hip).
hipError_t sort_pairs(uint32_t* key_in, uint32_t* key_out, uint32_t* val_in, uint32_t* val_out, int64_t n,
                      int bits, void* tmp, size_t* tmp_bytes, hipStream_t st);

}  // namespace tsmg
