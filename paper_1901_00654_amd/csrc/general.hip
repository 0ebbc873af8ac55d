// Kernels of the general form of the smoother (Sec. 2.1: degree q_p and
// knot intervals N_p per dimension; Sec. 3.2.1: the hierarchy halves every
// dimension), used when the problem is not cubic on equal power-of-two grids.
// They trade the tiled, register-blocked layout of the cubic kernels for
// generality: one thread per point evaluates its (q_p + 1) B-spline values
// per dimension by the uniform de Boor recursion and walks its
// prod_p (q_p + 1) patch entries; Lambda is applied one dimension at a time
// by banded passes of width 2 q_p + 1 (Alg. 2); the transfers are the
// per-dimension subdivision matrices of degree q_p (eq. 2.5).
#include "general.h"

namespace tsmg {

// B-splines of degree q alive on a knot interval, at u in [0, 1] of that
// interval (uniform knots, unit spacing): b[j] for the basis functions
// c - q + j... of the interval's first index c, i.e. b[0] is the one that
// ends at the interval's right knot. de Boor's recursion
//   b^k_j = ((u + k - j) b^{k-1}_{j-1} + (j + 1 - u) b^{k-1}_j) / k,
// with b^{k-1}_{-1} = b^{k-1}_k = 0, unrolled to kQMax with run-time guards
// so that the values stay in registers.
template <typename T>
__device__ __forceinline__ void bspline_values(T u, int q, T (&b)[kQMax + 1]) {
  b[0] = T(1);
#pragma unroll
  for (int j = 1; j <= kQMax; ++j) b[j] = T(0);
#pragma unroll
  for (int k = 1; k <= kQMax; ++k) {
    if (k <= q) {
      const T inv = T(1) / T(k);
      T prev = T(0);
#pragma unroll
      for (int j = 0; j <= kQMax; ++j) {
        if (j <= k) {
          const T cur = (j < k) ? b[j] : T(0);
          b[j] = ((u + T(k - j)) * prev + (T(j + 1) - u) * cur) * inv;
          prev = cur;
        }
      }
    }
  }
}

// b[a] for a run-time a in 0..kQMax without indexing the array at run time.
template <typename T>
__device__ __forceinline__ T pick(const T (&b)[kQMax + 1], int a) {
  T v = b[0];
#pragma unroll
  for (int m = 1; m <= kQMax; ++m) v = (a == m) ? b[m] : v;
  return v;
}

// Level cell and position of point i in dimension p (from its finest cell
// and the position inside it), and its B-spline values there.
template <typename T>
__device__ __forceinline__ int level_basis(const GenPoints& pts, const GenLevel& L, int p, int64_t i,
                                           T (&b)[kQMax + 1]) {
  const int cf = pts.cellp[size_t(p) * size_t(pts.n) + size_t(i)];
  const T t = static_cast<const T*>(pts.t)[size_t(p) * size_t(pts.n) + size_t(i)];
  const int sh = L.shift;
  const int cg = cf >> sh;
  const T u = (T(cf & ((1 << sh) - 1)) + t) * (T(1) / T(1 << sh));
  bspline_values<T>(u, L.q[p], b);
  return cg;
}

// out += Phi_g'(Phi_g c) (kApply), Phi_g'y (kRhs) or diag(Phi_g'Phi_g)
// (kDiag), one thread per point. The patch entries are walked as an
// odometer over the d digits (no divisions per entry). Points are sorted by
// their finest cell, so neighbouring lanes of a wave often share a level-g
// cell and hence every patch entry: before each entry's atomic, the lanes of
// such a run add their contributions by a segmented shuffle reduction and
// only the run's first lane adds the sum to the output.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_data_gen(GenPoints pts, GenLevel L, const T* c, T* out) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const bool live = i < pts.n;   // every lane takes part in the shuffles
  const int d = L.d;
  T b[kMaxDim][kQMax + 1];
  int64_t base = -1 - int64_t(threadIdx.x & 63);   // distinct for lanes past the end
  int P = 1;
  if (live) {
    base = 0;
#pragma unroll
    for (int p = 0; p < kMaxDim; ++p) {
      if (p < d) {
        const int cg = level_basis<T>(pts, L, p, i, b[p]);
        base += int64_t(cg) * L.stride[p];
        P *= L.q[p] + 1;
      }
    }
  } else {
#pragma unroll
    for (int p = 0; p < kMaxDim; ++p)
#pragma unroll
      for (int m = 0; m <= kQMax; ++m) b[p][m] = T(0);
  }
  // entry e as digits a[p]: index idx = base + sum_p a[p] stride[p]
  auto walk = [&](auto&& body) {
    int a[kMaxDim];
#pragma unroll
    for (int p = 0; p < kMaxDim; ++p) a[p] = 0;
    int64_t idx = base;
    for (int e = 0; e < P; ++e) {
      T w = T(1);
#pragma unroll
      for (int p = 0; p < kMaxDim; ++p)
        if (p < d) w *= pick<T>(b[p], a[p]);
      body(idx, w);
#pragma unroll
      for (int p = kMaxDim - 1; p >= 0; --p) {
        if (p >= d) continue;
        if (a[p] < L.q[p]) {
          ++a[p];
          idx += L.stride[p];
          break;
        }
        idx -= int64_t(a[p]) * L.stride[p];
        a[p] = 0;
      }
    }
  };
  T s = T(0);
  if constexpr (MODE == kApply) {
    if (live) walk([&](int64_t idx, T w) { s += w * c[idx]; });
  } else if constexpr (MODE == kRhs) {
    if (live) s = T(pts.y[i]);
  }
  // runs of lanes with the same level-g cell (the same patch)
  const int lane = threadIdx.x & 63;
  const int64_t prev = __shfl_up(base, 1);
  const bool head = lane == 0 || prev != base;
  const unsigned long long heads = __ballot(head);
  const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
  const int seg_end = above ? __ffsll(static_cast<long long>(above)) - 1 : 64;
  // the longest run in the wave bounds the reduction steps (uniform)
  int steps = 0;
  {
    int run = seg_end - lane;
    for (int o = 1; o < 64; o <<= 1) {
      const int r = __shfl_xor(run, o);
      run = run > r ? run : r;
    }
    while ((1 << steps) < run) ++steps;
  }
  // P is uniform over the live lanes; lanes past the end walk the same
  // number of entries with zero contributions
  int Pw = P;
  for (int o = 1; o < 64; o <<= 1) {
    const int r = __shfl_xor(Pw, o);
    Pw = Pw > r ? Pw : r;
  }
  P = Pw;
  walk([&](int64_t idx, T w) {
    T v = live ? (MODE == kDiag ? w * w : s * w) : T(0);
    for (int k = 0; k < steps; ++k) {
      const int o = 1 << k;
      const T u = __shfl_down(v, o);
      if (lane + o < seg_end) v += u;
    }
    if (head && live) atomicAdd(&out[idx], v);
  });
}

// One dimension p of the three-accumulator recursion for Lambda (Alg. 2):
//   T2' = M T2 + G2 T0 + 2 G1 T1,  T1' = M T1 + G1 T0,  T0' = M T0
// along dimension p (first pass: T0 = c, T1 = T2 = 0; last pass:
// out = lam T2'). band: [3][J][2q + 1], row j column j + o - q.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lambda_pass_gen(GenLambdaArgs<T> a) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= a.K) return;
  const int64_t inner = a.stride;
  const int j = int((k / inner) % a.J);
  const int64_t kb = k - int64_t(j) * inner;
  const int W = 2 * a.q + 1;
  const T* M = a.band;
  const T* G1 = a.band + size_t(a.J) * W;
  const T* G2 = a.band + 2 * size_t(a.J) * W;
  T s0 = T(0), s1 = T(0), s2 = T(0);
  const int l0 = j - a.q < 0 ? 0 : j - a.q;
  const int l1 = j + a.q > a.J - 1 ? a.J - 1 : j + a.q;
  for (int l = l0; l <= l1; ++l) {
    const size_t bi = size_t(j) * W + (l - j + a.q);
    const int64_t src = kb + int64_t(l) * inner;
    const T t0 = a.in0[src];
    if (a.first) {
      s0 += M[bi] * t0;
      s1 += G1[bi] * t0;
      s2 += G2[bi] * t0;
    } else {
      const T t1 = a.in1[src], t2 = a.in2[src];
      s0 += M[bi] * t0;
      s1 += M[bi] * t1 + G1[bi] * t0;
      s2 += M[bi] * t2 + G2[bi] * t0 + T(2) * G1[bi] * t1;
    }
  }
  if (a.last) {
    a.out[k] = a.lam * s2;
  } else {
    a.out0[k] = s0;
    a.out1[k] = s1;
    a.out2[k] = s2;
  }
}

// out[k] += lam * diag(Lambda)[k]: sum_p G2_p M.. + 2 sum_{p<q} G1_p G1_q M..
// from the centre entries of the banded factors.
__global__ __launch_bounds__(kBlock) void k_lambda_diag_gen(GenLevel L, const double* band, double lam,
                                                            double* out) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= L.K) return;
  double m[kMaxDim], g1[kMaxDim], g2[kMaxDim];
  int64_t rem = k;
  for (int p = L.d - 1; p >= 0; --p) {
    const int j = int(rem % L.J[p]);
    rem /= L.J[p];
    const int W = 2 * L.q[p] + 1;
    const double* bp = band + L.band_off[p];
    const size_t c = size_t(j) * W + L.q[p];
    m[p] = bp[c];
    g1[p] = bp[size_t(L.J[p]) * W + c];
    g2[p] = bp[2 * size_t(L.J[p]) * W + c];
  }
  double s = 0.0;
  for (int p = 0; p < L.d; ++p) {
    double t = g2[p];
    for (int r = 0; r < L.d; ++r)
      if (r != p) t *= m[r];
    s += t;
    for (int q = p + 1; q < L.d; ++q) {
      double u = 2.0 * g1[p] * g1[q];
      for (int r = 0; r < L.d; ++r)
        if (r != p && r != q) u *= m[r];
      s += u;
    }
  }
  out[k] += lam * s;
}

// binom(q + 1, m) / 2^q, the subdivision weights of degree q (eq. 2.5).
__device__ __forceinline__ double subdiv_weight(int q, int m) {
  if (m < 0 || m > q + 1) return 0.0;
  double c = 1.0;
  for (int i = 0; i < m; ++i) c = c * double(q + 1 - i) / double(i + 1);
  return c / double(1 << q);
}

// One dimension of the prolongation: out[o][i][r] (= or -=) sum_j
// I[i][j] in[o][j][r], I[i][j] = binom(q+1, i - 2j + q) / 2^q (0-based;
// fine functions outside the coarse range are absent, reading R3).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong_pass_gen(GenTransferArgs<T> a) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= a.Kout) return;
  const int64_t r = k % a.inner;
  const int i = int((k / a.inner) % a.Jf);
  const int64_t o = k / (a.inner * a.Jf);
  double s = 0.0;
  // j with 0 <= i - 2j + q <= q + 1
  int j0 = (i - 1 + 1) / 2;   // ceil((i - 1) / 2) for i >= 0
  if (i == 0) j0 = 0;
  const int j1 = (i + a.q) / 2;
  for (int j = j0; j <= j1; ++j) {
    if (j < 0 || j >= a.Jc) continue;
    s += subdiv_weight(a.q, i - 2 * j + a.q) * double(a.in[(o * a.Jc + j) * a.inner + r]);
  }
  if (a.subtract) a.out[k] -= T(s);
  else a.out[k] = T(s);
}

// One dimension of the restriction (the transposed prolongation):
// out[o][j][r] = sum_i I[i][j] (in - sub)[o][i][r], i = 2j - q + m, m = 0..q+1.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_pass_gen(GenTransferArgs<T> a) {
  const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (k >= a.Kout) return;
  const int64_t r = k % a.inner;
  const int j = int((k / a.inner) % a.Jc);
  const int64_t o = k / (a.inner * a.Jc);
  double s = 0.0;
  for (int m = 0; m <= a.q + 1; ++m) {
    const int i = 2 * j - a.q + m;
    if (i < 0 || i >= a.Jf) continue;
    const int64_t src = (o * a.Jf + i) * a.inner + r;
    const double v = a.sub ? double(a.in[src]) - double(a.sub[src]) : double(a.in[src]);
    s += subdiv_weight(a.q, m) * v;
  }
  a.out[k] = T(s);
}

// Dense coarse matrix (Sec. 3.2.4): A += lam Lambda, one thread per entry,
// from the banded 1D factors (A zeroed first).
__global__ __launch_bounds__(kBlock) void k_dense_lambda_gen(GenLevel L, const double* band, double lam, double* A) {
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= L.K * L.K) return;
  const int64_t k = t / L.K, l = t % L.K;
  double m[kMaxDim], g1[kMaxDim], g2[kMaxDim];
  int64_t rk = k, rl = l;
  for (int p = L.d - 1; p >= 0; --p) {
    const int jk = int(rk % L.J[p]), jl = int(rl % L.J[p]);
    rk /= L.J[p];
    rl /= L.J[p];
    const int o = jl - jk;
    if (o < -L.q[p] || o > L.q[p]) return;   // outside every band: zero
    const int W = 2 * L.q[p] + 1;
    const double* bp = band + L.band_off[p];
    const size_t c = size_t(jk) * W + (o + L.q[p]);
    m[p] = bp[c];
    g1[p] = bp[size_t(L.J[p]) * W + c];
    g2[p] = bp[2 * size_t(L.J[p]) * W + c];
  }
  double s = 0.0;
  for (int p = 0; p < L.d; ++p) {
    double tt = g2[p];
    for (int r = 0; r < L.d; ++r)
      if (r != p) tt *= m[r];
    s += tt;
    for (int q = p + 1; q < L.d; ++q) {
      double u = 2.0 * g1[p] * g1[q];
      for (int r = 0; r < L.d; ++r)
        if (r != p && r != q) u *= m[r];
      s += u;
    }
  }
  A[t] += lam * s;
}

// Dense coarse matrix: A += Phi'Phi, one thread per (point, patch entry a),
// adding phi_a phi_b for every patch entry b; the lanes of a wave that share
// a cell (and so the row a) sum their terms by shuffles before one atomic.
__global__ __launch_bounds__(kBlock) void k_dense_gram_gen(GenPoints pts, GenLevel L, int P, double* A) {
  // thread t: patch entry ea = t / n of point i = t % n, so that the lanes of
  // a wave are consecutive points with the same ea
  const int64_t t = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  const bool live = t < pts.n * int64_t(P);
  const int64_t i = live ? t % pts.n : 0;
  const int ea = live ? int(t / pts.n) : 0;
  const int d = L.d;
  double b[kMaxDim][kQMax + 1];
  int64_t base = 0;
#pragma unroll
  for (int p = 0; p < kMaxDim; ++p) {
    if (p < d) base += int64_t(level_basis<double>(pts, L, p, i, b[p])) * L.stride[p];
  }
  auto entry = [&](int e, int64_t& idx) {
    int rem = e;
    idx = base;
    double w = 1.0;
#pragma unroll
    for (int p = kMaxDim - 1; p >= 0; --p) {
      if (p < d) {
        const int a = rem % (L.q[p] + 1);
        rem /= L.q[p] + 1;
        w *= pick<double>(b[p], a);
        idx += int64_t(a) * L.stride[p];
      }
    }
    return w;
  };
  int64_t ka;
  double wa = entry(ea, ka);
  if (!live) {
    wa = 0.0;
    ka = -1 - int64_t(threadIdx.x & 63);   // a run of its own
  }
  // runs of lanes with the same row ka (the same cell and entry): their
  // contributions to every A[ka][kb] are summed by shuffles first
  const int lane = threadIdx.x & 63;
  const int64_t prev = __shfl_up(ka, 1);
  const bool head = lane == 0 || prev != ka;
  const unsigned long long heads = __ballot(head);
  const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
  const int seg_end = above ? __ffsll(static_cast<long long>(above)) - 1 : 64;
  int steps = 0;
  {
    int run = seg_end - lane;
    for (int o = 1; o < 64; o <<= 1) {
      const int r = __shfl_xor(run, o);
      run = run > r ? run : r;
    }
    while ((1 << steps) < run) ++steps;
  }
  for (int eb = 0; eb < P; ++eb) {
    int64_t kb;
    const double wb = entry(eb, kb);
    double v = wa * wb;
    for (int k = 0; k < steps; ++k) {
      const int o = 1 << k;
      const double u = __shfl_down(v, o);
      if (lane + o < seg_end) v += u;
    }
    if (head && live) atomicAdd(&A[ka * L.K + kb], v);
  }
}

// Finest cell of every point (C order over the per-dimension cells) and the
// validity flags (bit 2: non-finite x, bit 4: outside the box).
__global__ __launch_bounds__(kBlock) void k_bin_gen(const double* x, int64_t n, GenBox box, uint32_t* key,
                                                    uint32_t* idx, int* flag) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= n) return;
  uint32_t k = 0;
  int bad = 0;
  for (int p = 0; p < box.d; ++p) {
    const double xv = x[size_t(i) * box.d + p];
    int64_t ci = 0;
    if (!isfinite(xv)) bad |= 2;
    else if (xv < box.lo[p] || xv > box.hi[p]) bad |= 4;
    else {
      ci = int64_t(floor((xv - box.lo[p]) * box.inv_h[p]));
      ci = ci < 0 ? 0 : (ci > box.N[p] - 1 ? box.N[p] - 1 : ci);
    }
    k = k * uint32_t(box.N[p]) + uint32_t(ci);
  }
  key[i] = k;
  idx[i] = uint32_t(i);
  if (bad) atomicOr(flag, bad);
}

// Sorted points to structure-of-arrays storage: per dimension the finest
// cell and the position inside it (FP64 and FP32), and the responses.
__global__ __launch_bounds__(kBlock) void k_place_gen(const double* x, const double* y, const uint32_t* idx,
                                                      int64_t n, GenBox box, int32_t* cellp, double* t64, float* t32,
                                                      double* ys) {
  const int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (s >= n) return;
  const int64_t i = idx[s];
  for (int p = 0; p < box.d; ++p) {
    const double u = (x[size_t(i) * box.d + p] - box.lo[p]) * box.inv_h[p];
    int64_t ci = int64_t(floor(u));
    ci = ci < 0 ? 0 : (ci > box.N[p] - 1 ? box.N[p] - 1 : ci);
    double t = u - double(ci);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
    cellp[size_t(p) * n + s] = int32_t(ci);
    t64[size_t(p) * n + s] = t;
    t32[size_t(p) * n + s] = float(t);
  }
  ys[s] = y[i];
}

// s(x) at query points (eq. 2.2) on the finest level; queries outside the
// box are evaluated on the polynomial piece of the nearest boundary cell.
__global__ __launch_bounds__(kBlock) void k_eval_gen(const double* alpha, const double* xq, int64_t m, GenBox box,
                                                     GenLevel L, double* yq) {
  const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= m) return;
  const int d = L.d;
  double b[kMaxDim][kQMax + 1];
  int64_t base = 0;
  int P = 1;
#pragma unroll
  for (int p = 0; p < kMaxDim; ++p) {
    if (p < d) {
      const double u = (xq[size_t(i) * d + p] - box.lo[p]) * box.inv_h[p];
      double fl = floor(u);
      fl = fl < 0.0 ? 0.0 : (fl > double(box.N[p] - 1) ? double(box.N[p] - 1) : fl);
      bspline_values<double>(u - fl, L.q[p], b[p]);
      base += int64_t(fl) * L.stride[p];
      P *= L.q[p] + 1;
    }
  }
  double s = 0.0;
  for (int e = 0; e < P; ++e) {
    int rem = e;
    int64_t idx = base;
    double w = 1.0;
#pragma unroll
    for (int p = kMaxDim - 1; p >= 0; --p) {
      if (p < d) {
        const int a = rem % (L.q[p] + 1);
        rem /= L.q[p] + 1;
        w *= pick<double>(b[p], a);
        idx += int64_t(a) * L.stride[p];
      }
    }
    s += w * alpha[idx];
  }
  yq[i] = s;
}

// ---------------------------------------------------------------------------
static inline unsigned blocks_for_gen(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

template <typename T>
hipError_t launch_data_gen(int mode, const GenPoints& pts, const GenLevel& L, const T* c, T* out, hipStream_t st) {
  if (pts.n == 0) return hipSuccess;
  const unsigned g = blocks_for_gen(pts.n);
  if (mode == kApply) hipLaunchKernelGGL((k_data_gen<T, kApply>), dim3(g), dim3(kBlock), 0, st, pts, L, c, out);
  else if (mode == kRhs) hipLaunchKernelGGL((k_data_gen<T, kRhs>), dim3(g), dim3(kBlock), 0, st, pts, L, c, out);
  else hipLaunchKernelGGL((k_data_gen<T, kDiag>), dim3(g), dim3(kBlock), 0, st, pts, L, c, out);
  return hipGetLastError();
}
template hipError_t launch_data_gen<double>(int, const GenPoints&, const GenLevel&, const double*, double*,
                                            hipStream_t);
template hipError_t launch_data_gen<float>(int, const GenPoints&, const GenLevel&, const float*, float*,
                                           hipStream_t);

template <typename T>
hipError_t launch_lambda_pass_gen(const GenLambdaArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL(k_lambda_pass_gen<T>, dim3(blocks_for_gen(a.K)), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_lambda_pass_gen<double>(const GenLambdaArgs<double>&, hipStream_t);
template hipError_t launch_lambda_pass_gen<float>(const GenLambdaArgs<float>&, hipStream_t);

hipError_t launch_lambda_diag_gen(const GenLevel& L, const double* band, double lam, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_lambda_diag_gen, dim3(blocks_for_gen(L.K)), dim3(kBlock), 0, st, L, band, lam, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transfer_gen(bool prolong, const GenTransferArgs<T>& a, hipStream_t st) {
  if (prolong) hipLaunchKernelGGL(k_prolong_pass_gen<T>, dim3(blocks_for_gen(a.Kout)), dim3(kBlock), 0, st, a);
  else hipLaunchKernelGGL(k_restrict_pass_gen<T>, dim3(blocks_for_gen(a.Kout)), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}
template hipError_t launch_transfer_gen<double>(bool, const GenTransferArgs<double>&, hipStream_t);
template hipError_t launch_transfer_gen<float>(bool, const GenTransferArgs<float>&, hipStream_t);

hipError_t launch_dense_coarse_gen(const GenPoints& pts, const GenLevel& L, const double* band, double lam,
                                   double* A, hipStream_t st) {
  hipLaunchKernelGGL(k_dense_lambda_gen, dim3(blocks_for_gen(L.K * L.K)), dim3(kBlock), 0, st, L, band, lam, A);
  int P = 1;
  for (int p = 0; p < L.d; ++p) P *= L.q[p] + 1;
  if (pts.n > 0)
    hipLaunchKernelGGL(k_dense_gram_gen, dim3(blocks_for_gen(pts.n * int64_t(P))), dim3(kBlock), 0, st, pts, L, P,
                       A);
  return hipGetLastError();
}

hipError_t launch_bin_gen(const double* x, int64_t n, const GenBox& box, uint32_t* key, uint32_t* idx, int* flag,
                          hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin_gen, dim3(blocks_for_gen(n)), dim3(kBlock), 0, st, x, n, box, key, idx, flag);
  return hipGetLastError();
}

hipError_t launch_place_gen(const double* x, const double* y, const uint32_t* idx, int64_t n, const GenBox& box,
                            int32_t* cellp, double* t64, float* t32, double* ys, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_place_gen, dim3(blocks_for_gen(n)), dim3(kBlock), 0, st, x, y, idx, n, box, cellp, t64, t32,
                     ys);
  return hipGetLastError();
}

hipError_t launch_eval_gen(const double* alpha, const double* xq, int64_t m, const GenBox& box, const GenLevel& L,
                           double* yq, hipStream_t st) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_gen, dim3(blocks_for_gen(m)), dim3(kBlock), 0, st, alpha, xq, m, box, L, yq);
  return hipGetLastError();
}

}  // namespace tsmg
