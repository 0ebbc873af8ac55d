// Launch interface of the general-form kernels (general.hip): B-spline
// degree q_p and knot intervals N_p per dimension (Sec. 2.1).
#pragma once
#include "common.h"

namespace tsmg {

constexpr int kQMax = 5;   // highest B-spline degree of the general form

// The box and finest grid of a general problem.
struct GenBox {
  int d;
  int N[kMaxDim];          // finest intervals per dimension
  double lo[kMaxDim];
  double hi[kMaxDim];
  double inv_h[kMaxDim];   // N_p / (hi_p - lo_p)
};

// One level g: N_{g,p} = N_p / 2^(G-g) intervals, J_{g,p} = N_{g,p} + q_p
// coefficients per dimension, C-order strides.
struct GenLevel {
  int d;
  int N[kMaxDim];
  int J[kMaxDim];
  int q[kMaxDim];
  int shift;                  // G - g: finest cell index -> level-g cell index
  int64_t stride[kMaxDim];    // prod_{r > p} J_r
  int64_t K;
  int64_t band_off[kMaxDim];  // offset of dimension p's [3][J_p][2 q_p + 1] factors
};

// Sorted points of a general problem (structure of arrays).
struct GenPoints {
  int64_t n;
  const int32_t* cellp;   // [d][n] finest cell per dimension
  const void* t;          // [d][n] T: position inside that cell, in [0, 1]
  const double* y;        // [n] responses
};

template <typename T>
struct GenLambdaArgs {
  const T* in0; const T* in1; const T* in2;   // T0, T1, T2 (in1/in2 unused when first)
  T* out0; T* out1; T* out2;                  // next T0, T1, T2 (unused when last)
  T* out;                                     // lam * T2 (last pass only)
  const T* band;                              // [3][J][2q + 1]: M, G1, G2 of this dimension
  int64_t K;                                  // entries of the tensor
  int64_t stride;                             // product of the sizes after this dimension
  int J, q;
  int first, last;
  T lam;
};

template <typename T>
struct GenTransferArgs {
  const T* in;
  T* out;
  int64_t Kout;
  int64_t inner;    // product of the sizes of the dimensions after p
  int Jc, Jf, q;    // coarse / fine length and degree of dimension p
  int subtract;     // prolongation only: out -= value
  const T* sub;     // restriction only: input is in - sub (null: in)
};

template <typename T>
hipError_t launch_data_gen(int mode, const GenPoints& pts, const GenLevel& L, const T* c, T* out, hipStream_t st);
template <typename T> hipError_t launch_lambda_pass_gen(const GenLambdaArgs<T>& a, hipStream_t st);
hipError_t launch_lambda_diag_gen(const GenLevel& L, const double* band, double lam, double* out, hipStream_t st);
template <typename T> hipError_t launch_transfer_gen(bool prolong, const GenTransferArgs<T>& a, hipStream_t st);
// A += lam Lambda_c + Phi_c'Phi_c, dense K x K (A zeroed by the caller).
hipError_t launch_dense_coarse_gen(const GenPoints& pts, const GenLevel& L, const double* band, double lam,
                                   double* A, hipStream_t st);
hipError_t launch_bin_gen(const double* x, int64_t n, const GenBox& box, uint32_t* key, uint32_t* idx, int* flag,
                          hipStream_t st);
hipError_t launch_place_gen(const double* x, const double* y, const uint32_t* idx, int64_t n, const GenBox& box,
                            int32_t* cellp, double* t64, float* t32, double* ys, hipStream_t st);
hipError_t launch_eval_gen(const double* alpha, const double* xq, int64_t m, const GenBox& box, const GenLevel& L,
                           double* yq, hipStream_t st);

}  // namespace tsmg
