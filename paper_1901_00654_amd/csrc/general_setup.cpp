// Host side of the general form: B-spline degree q_p and knot intervals N_p
// per dimension (Sec. 2.1), any N_p >= 1, the hierarchy halving every
// dimension while all N_p are even (Sec. 3.2.1, eq. 2.5 per dimension).
// Setup bins and sorts the points by their finest cell in C order, builds
// the banded 1D Gram factors of every level exactly, and the operators
// apply the general kernels (general.hip) matrix-free on every level.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "general.h"
#include "problem.h"

namespace tsmg {

bool needs_general(int d, int q, const int32_t* N, const int32_t* degrees) {
  for (int p = 0; p < d; ++p) {
    const int qp = degrees ? degrees[p] : q;
    if (qp != kDeg || N[p] != N[0] || N[p] < 2 || (N[p] & (N[p] - 1)) != 0) return true;
  }
  return false;
}

int general_levels(int d, const int32_t* N) {
  std::vector<int> Ns(N, N + d);
  int G = 1;
  for (;;) {
    bool even = true, all2 = true;
    for (int v : Ns) {
      even = even && (v % 2 == 0);
      all2 = all2 && (v == 2);
    }
    if (!even || all2) break;
    for (int& v : Ns) v /= 2;
    ++G;
  }
  return G;
}

int64_t footprint_general(int d, int q, const int32_t* N, int64_t n, const ts_options& opt) {
  const int G = general_levels(d, N);
  const int c = std::max(1, std::min(G, opt.coarsest_level));
  int64_t levels = 0, KG = 0, Kc = 0;
  for (int g = c; g <= G; ++g) {
    int64_t K = 1;
    for (int p = 0; p < d; ++p) K *= (N[p] >> (G - g)) + (opt.degrees ? opt.degrees[p] : q);
    levels += 56 * K;
    if (g == G) KG = K;
    if (g == c) Kc = K;
  }
  const int64_t points = n * (16 * int64_t(d) + 8) + 24 * n + (1 << 20);   // sorted points, sort temporaries
  const int64_t finest = KG * (6 * 12 + 2 * 12 + 5 * 8 + 5 * 4 + 8);
  const int64_t coarse = opt.coarse_solver == TS_COARSE_CG ? 6 * Kc * 8 : 2 * Kc * Kc * 8 + 2 * Kc * 8;
  // the dense V-cycle operator of the lower levels and its assembly
  std::vector<int64_t> Kl(size_t(G) + 1, 0);
  std::vector<char> ok(size_t(G) + 1, 1);
  for (int g = c; g <= G; ++g) {
    int64_t K = 1;
    for (int p = 0; p < d; ++p) K *= (N[p] >> (G - g)) + (opt.degrees ? opt.degrees[p] : q);
    Kl[size_t(g)] = K;
  }
  const int gb = choose_bottom(opt, c, G, Kl, ok, true);
  int64_t bottom = 0;
  for (int g = c + 1; g <= gb; ++g) {
    const int64_t Kf = Kl[size_t(g)], Kg = Kl[size_t(g) - 1];
    bottom = std::max(bottom, (5 * Kf * Kf + 6 * Kg * Kf + 2 * Kg * Kg) * 8);
  }
  if (gb > 0) bottom += Kl[size_t(gb)] * Kl[size_t(gb)] * 12;
  return points + levels + finest + coarse + bottom + int64_t(64) * 4096 * (G + 2);
}

namespace {

// Polynomial (coefficients of u^0..u^q) of each of the q + 1 B-splines of
// degree q alive on a unit interval, in the order of bspline_values (de
// Boor's recursion carried out on polynomials).
std::vector<std::vector<double>> local_pieces(int q) {
  std::vector<std::vector<double>> b(1, std::vector<double>(1, 1.0));
  for (int k = 1; k <= q; ++k) {
    std::vector<std::vector<double>> nb(size_t(k) + 1, std::vector<double>(size_t(k) + 1, 0.0));
    for (int j = 0; j <= k; ++j) {
      // ((u + k - j) b_{j-1} + (j + 1 - u) b_j) / k
      if (j - 1 >= 0) {
        const auto& pv = b[size_t(j) - 1];
        for (size_t e = 0; e < pv.size(); ++e) {
          nb[size_t(j)][e + 1] += pv[e] / k;
          nb[size_t(j)][e] += pv[e] * double(k - j) / k;
        }
      }
      if (j < k) {
        const auto& cv = b[size_t(j)];
        for (size_t e = 0; e < cv.size(); ++e) {
          nb[size_t(j)][e] += cv[e] * double(j + 1) / k;
          nb[size_t(j)][e + 1] -= cv[e] / k;
        }
      }
    }
    b.swap(nb);
  }
  return b;
}

std::vector<double> derive(const std::vector<double>& c, int r) {
  std::vector<double> v = c;
  for (int k = 0; k < r; ++k) {
    for (size_t i = 0; i + 1 < v.size(); ++i) v[i] = v[i + 1] * double(i + 1);
    if (!v.empty()) v.back() = 0.0;
  }
  return v;
}

// Banded 1D Gram factors of degree q on [lo, hi] with N intervals (Sec. 2.4):
// band[r][j][o] = int D^r B_j D^r B_{j + o - q} over the box, o = 0..2q,
// each interval's (q+1) x (q+1) block integrated exactly in the local
// coordinate and scaled by h^(1 - 2r).
void gram_band_general(double lo, double hi, int N, int q, std::vector<double>& band) {
  const int J = N + q, W = 2 * q + 1;
  const double h = (hi - lo) / N;
  const auto pieces = local_pieces(q);
  band.assign(size_t(3) * J * W, 0.0);
  for (int r = 0; r < 3; ++r) {
    std::vector<std::vector<double>> loc(size_t(q) + 1, std::vector<double>(size_t(q) + 1, 0.0));
    for (int a = 0; a <= q; ++a)
      for (int b = 0; b <= q; ++b) {
        const auto pa = derive(pieces[size_t(a)], r), pb = derive(pieces[size_t(b)], r);
        double s = 0.0;
        for (size_t i = 0; i < pa.size(); ++i)
          for (size_t j = 0; j < pb.size(); ++j) s += pa[i] * pb[j] / double(i + j + 1);
        loc[size_t(a)][size_t(b)] = s * std::pow(h, 1.0 - 2.0 * r);
      }
    for (int c = 0; c < N; ++c)
      for (int a = 0; a <= q; ++a)
        for (int b = 0; b <= q; ++b)
          band[(size_t(r) * J + size_t(c + a)) * W + size_t(b - a + q)] += loc[size_t(a)][size_t(b)];
  }
}

GenPoints points_of(Problem* P, bool fp32) {
  GenPoints pts{};
  pts.n = P->n;
  pts.cellp = P->gcell.p;
  pts.t = fp32 ? static_cast<const void*>(P->t32.p) : static_cast<const void*>(P->t64.p);
  pts.y = P->ys.p;
  return pts;
}

template <typename T> const T* gband(Level& L);
template <> const double* gband<double>(Level& L) { return L.band64.p; }
template <> const float* gband<float>(Level& L) { return L.band32.p; }
template <typename T> T* glam(Problem* P);
template <> double* glam<double>(Problem* P) { return P->lamS64.p; }
template <> float* glam<float>(Problem* P) { return P->lamS32.p; }
template <typename T> T* gxfer(Problem* P);
template <> double* gxfer<double>(Problem* P) { return P->xfer64.p; }
template <> float* gxfer<float>(Problem* P) { return P->xfer32.p; }

}  // namespace

void setup_general_points(Problem* P, const int32_t* N, const int32_t* q, const double* lo, const double* hi,
                          const double* x, const double* y) {
  const int d = P->d;
  const int64_t n = P->n;
  hipStream_t st = P->stream;
  GenBox& B = P->gbox;
  B.d = d;
  int64_t ncells = 1;
  for (int p = 0; p < d; ++p) {
    B.N[p] = N[p];
    B.lo[p] = lo[p];
    B.hi[p] = hi[p];
    B.inv_h[p] = double(N[p]) / (hi[p] - lo[p]);
    P->gq[p] = q[p];
    ncells *= N[p];
  }
  int bits = 1;
  while ((int64_t(1) << bits) < ncells) ++bits;
  DevBuf<uint32_t> key0, key1, idx0, idx1;
  key0.alloc(size_t(n));
  key1.alloc(size_t(n));
  idx0.alloc(size_t(n));
  idx1.alloc(size_t(n));
  hip_check(launch_fill<int>(P->flag.p, 0, 1, st), "fill");
  hip_check(launch_bin_gen(x, n, B, key0.p, idx0.p, P->flag.p, st), "bin");
  hip_check(launch_check_finite(y, n, P->flag.p, st), "check y");
  int flag = 0;
  hip_check(hipMemcpyAsync(&flag, P->flag.p, sizeof(int), hipMemcpyDeviceToHost, st), "flag");
  hip_check(hipStreamSynchronize(st), "sync");
  if (flag & 2) throw Error{TS_EINVAL, "x contains non-finite values"};
  if (flag & 4) throw Error{TS_EINVAL, "some points lie outside [lo, hi]"};
  if (flag & 1) throw Error{TS_EINVAL, "y contains non-finite values"};
  size_t tmp_bytes = 0;
  hip_check(sort_pairs(key0.p, key1.p, idx0.p, idx1.p, n, bits, nullptr, &tmp_bytes, st), "sort size");
  DevBuf<unsigned char> tmp;
  tmp.alloc(tmp_bytes + 16);
  hip_check(sort_pairs(key0.p, key1.p, idx0.p, idx1.p, n, bits, tmp.p, &tmp_bytes, st), "sort");
  P->t64.alloc(size_t(n) * d);
  P->t32.alloc(size_t(n) * d);
  P->gcell.alloc(size_t(n) * d);
  P->ys.alloc(size_t(n));
  hip_check(launch_place_gen(x, y, idx1.p, n, B, P->gcell.p, P->t64.p, P->t32.p, P->ys.p, st), "place");
  hip_check(hipStreamSynchronize(st), "sync");
}

void setup_general_level(Problem* P, int g, const double* lo, const double* hi) {
  Level& L = P->lev[g];
  GenLevel& gl = L.gl;
  const int d = P->d;
  gl.d = d;
  gl.shift = P->G - g;
  gl.K = 1;
  for (int p = 0; p < d; ++p) {
    gl.N[p] = P->gbox.N[p] >> gl.shift;
    gl.q[p] = P->gq[p];
    gl.J[p] = gl.N[p] + gl.q[p];
    gl.K *= gl.J[p];
  }
  for (int p = d - 1; p >= 0; --p) gl.stride[p] = (p == d - 1) ? 1 : gl.stride[p + 1] * gl.J[p + 1];
  L.g = g;
  L.K = gl.K;
  L.N = gl.N[0];
  L.J = gl.J[0];
  std::vector<double> band;
  for (int p = 0; p < d; ++p) {
    gl.band_off[p] = int64_t(band.size());
    std::vector<double> b1;
    gram_band_general(lo[p], hi[p], gl.N[p], gl.q[p], b1);
    band.insert(band.end(), b1.begin(), b1.end());
  }
  std::vector<float> bandf(band.begin(), band.end());
  L.band64.alloc(band.size());
  L.band32.alloc(band.size());
  hipStream_t st = P->stream;
  hip_check(hipMemcpyAsync(L.band64.p, band.data(), band.size() * 8, hipMemcpyHostToDevice, st), "upload");
  hip_check(hipMemcpyAsync(L.band32.p, bandf.data(), bandf.size() * 4, hipMemcpyHostToDevice, st), "upload");
  hip_check(hipStreamSynchronize(st), "sync");   // host band vectors go out of scope
}

// out = lambda Lambda_g c: one banded pass per dimension (Alg. 2).
template <typename T>
static void lambda_apply_general(Problem* P, int g, const T* c, T* out) {
  Level& L = P->lev[g];
  const GenLevel& gl = L.gl;
  const int d = P->d;
  T* S = glam<T>(P);
  T* bufA = S;
  T* bufB = S + 3 * P->lev[P->G].K;
  const T* in0 = c;
  const T* in1 = nullptr;
  const T* in2 = nullptr;
  for (int p = 0; p < d; ++p) {
    GenLambdaArgs<T> a{};
    a.in0 = in0; a.in1 = in1; a.in2 = in2;
    a.band = gband<T>(L) + gl.band_off[p];
    a.K = gl.K;
    a.stride = gl.stride[p];
    a.J = gl.J[p];
    a.q = gl.q[p];
    a.first = (p == 0);
    a.last = (p == d - 1);
    a.lam = T(P->lam);
    T* o = (p % 2 == 0) ? bufA : bufB;
    a.out0 = o; a.out1 = o + gl.K; a.out2 = o + 2 * gl.K;
    a.out = out;
    hip_check(launch_lambda_pass_gen<T>(a, P->stream), "lambda pass");
    in0 = a.out0; in1 = a.out1; in2 = a.out2;
  }
}

template <typename T>
void apply_general(Problem* P, int g, const T* c, T* out) {
  lambda_apply_general<T>(P, g, c, out);
  hip_check(launch_data_gen<T>(kApply, points_of(P, sizeof(T) == 4), P->lev[g].gl, c, out, P->stream), "data pass");
}
template void apply_general<double>(Problem*, int, const double*, double*);
template void apply_general<float>(Problem*, int, const float*, float*);

// Times `reps` launches of the Lambda passes and of the point pass.
template <typename T>
void profile_general(Problem* P, int g, T* c, T* out, int reps, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2) {
  hip_check(hipEventRecord(e0, P->stream), "record");
  for (int i = 0; i < reps; ++i) lambda_apply_general<T>(P, g, c, out);
  hip_check(hipEventRecord(e1, P->stream), "record");
  for (int i = 0; i < reps; ++i)
    hip_check(launch_data_gen<T>(kApply, points_of(P, sizeof(T) == 4), P->lev[g].gl, c, out, P->stream), "data");
  hip_check(hipEventRecord(e2, P->stream), "record");
}
template void profile_general<double>(Problem*, int, double*, double*, int, hipEvent_t, hipEvent_t, hipEvent_t);
template void profile_general<float>(Problem*, int, float*, float*, int, hipEvent_t, hipEvent_t, hipEvent_t);

// Prolongation (out = or -= I e) and restriction (out = I'(r - sub)) between
// levels g-1 and g, one subdivision pass per dimension.
template <typename T>
void transfer_general(Problem* P, int g, bool prolong, const T* in, T* out, const T* sub, bool subtract) {
  const GenLevel& F = P->lev[g].gl;
  const GenLevel& C = P->lev[g - 1].gl;
  const int d = P->d;
  T* X = gxfer<T>(P);
  T* bufs[2] = {X, X + P->lev[P->G].K};
  const T* cur = in;
  for (int p = 0; p < d; ++p) {
    GenTransferArgs<T> a{};
    int64_t inner = 1, outer = 1;
    for (int r = p + 1; r < d; ++r) inner *= prolong ? C.J[r] : F.J[r];
    for (int r = 0; r < p; ++r) outer *= prolong ? F.J[r] : C.J[r];
    a.in = cur;
    a.out = (p == d - 1) ? out : bufs[p % 2];
    a.Kout = outer * (prolong ? F.J[p] : C.J[p]) * inner;
    a.inner = inner;
    a.Jc = C.J[p];
    a.Jf = F.J[p];
    a.q = F.q[p];
    a.subtract = (prolong && p == d - 1 && subtract) ? 1 : 0;
    a.sub = (!prolong && p == 0) ? sub : nullptr;
    hip_check(launch_transfer_gen<T>(prolong, a, P->stream), prolong ? "prolongation" : "restriction");
    cur = a.out;
  }
}
template void transfer_general<double>(Problem*, int, bool, const double*, double*, const double*, bool);
template void transfer_general<float>(Problem*, int, bool, const float*, float*, const float*, bool);

void rhs_general(Problem* P, double* b) {
  hip_check(launch_fill<double>(b, 0.0, P->lev[P->G].K, P->stream), "fill");
  hip_check(launch_data_gen<double>(kRhs, points_of(P, false), P->lev[P->G].gl, nullptr, b, P->stream), "rhs");
}

void diag_general(Problem* P, int g) {
  Level& L = P->lev[g];
  hip_check(launch_fill<double>(L.diag.p, 0.0, L.K, P->stream), "fill");
  hip_check(launch_lambda_diag_gen(L.gl, L.band64.p, P->lam, L.diag.p, P->stream), "lambda diag");
  hip_check(launch_data_gen<double>(kDiag, points_of(P, false), L.gl, nullptr, L.diag.p, P->stream), "data diag");
}

void coarse_matrix_general(Problem* P, double* A) { dense_level_general(P, P->Gc, A); }

void dense_level_general(Problem* P, int g, double* A) {
  Level& L = P->lev[g];
  hip_check(launch_fill<double>(A, 0.0, L.K * L.K, P->stream), "fill");
  hip_check(launch_dense_coarse_gen(points_of(P, false), L.gl, L.band64.p, P->lam, A, P->stream), "dense level");
}

// R = I_g' (K_{g-1} x K_g): every coarse unit vector prolongated at once, one
// subdivision pass per dimension over a leading batch index (row j of R is
// I_g e_j, the j-th column of I_g).
void restriction_dense_general(Problem* P, int g, double* R) {
  const GenLevel& F = P->lev[g].gl;
  const GenLevel& C = P->lev[g - 1].gl;
  const int d = P->d;
  const int64_t Kc = C.K, Kf = F.K;
  hipStream_t st = P->stream;
  DevBuf<double> one, bufs[2];
  one.alloc(size_t(Kc));
  bufs[0].alloc(size_t(Kc * Kf));
  bufs[1].alloc(size_t(Kc * Kf));
  hip_check(launch_fill<double>(one.p, 1.0, Kc, st), "fill");
  hip_check(launch_diag_dense(one.p, Kc, bufs[0].p, st), "identity");
  const double* cur = bufs[0].p;
  for (int p = 0; p < d; ++p) {
    GenTransferArgs<double> a{};
    int64_t inner = 1, outer = Kc;
    for (int r = p + 1; r < d; ++r) inner *= C.J[r];
    for (int r = 0; r < p; ++r) outer *= F.J[r];
    a.in = cur;
    a.out = (p == d - 1) ? R : bufs[(p + 1) % 2].p;
    a.Kout = outer * F.J[p] * inner;
    a.inner = inner;
    a.Jc = C.J[p];
    a.Jf = F.J[p];
    a.q = F.q[p];
    hip_check(launch_transfer_gen<double>(true, a, st), "prolongation");
    cur = a.out;
  }
  hip_check(hipStreamSynchronize(st), "sync");   // the work buffers are released
}

void eval_general(Problem* P, const double* alpha, int64_t m, const double* xq, double* yq) {
  hip_check(launch_eval_gen(alpha, xq, m, P->gbox, P->lev[P->G].gl, yq, P->stream), "evaluate");
}

}  // namespace tsmg
