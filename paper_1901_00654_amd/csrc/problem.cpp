// Host side of tsmg: problem setup, the level hierarchy, the V-cycle (Alg. 7),
// PCG (Alg. 8), the mixed-precision refinement loop and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <future>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/tsmg.h"
#include "launch.h"
#include "problem.h"

namespace tsmg {

thread_local std::string g_last_error;
thread_local MemCount g_mem;

void set_error(const std::string& m) { g_last_error = m; }

// ---------------------------------------------------------------------------
// Device memory cache. Sizes are rounded up (64 KiB steps to 16 MiB, 2 MiB
// steps above) and a cached block is reused for a request of at least 4/5
// of its size. The cache holds at most min(8 GiB, 1/16 of the device) per
// device. It is never torn down: the blocks live until the process ends.
namespace {
struct DevicePool {
  std::multimap<size_t, void*> free_blocks;   // size -> block
  size_t cached = 0;
  size_t cap = 0;
};
struct Pool {
  std::mutex m;
  std::map<int, DevicePool> dev;
  std::unordered_map<void*, std::pair<int, size_t>> live;   // block -> (device, size)
};
Pool& pool() {
  static Pool* p = new Pool;   // not destroyed at exit: the runtime may be gone by then
  return *p;
}
size_t pool_round(size_t b) {
  const size_t q = b <= (size_t(16) << 20) ? (size_t(64) << 10) : (size_t(2) << 20);
  return (b + q - 1) / q * q;
}
}  // namespace

thread_local Arena* g_arena = nullptr;

namespace {
struct ArenaRegions {
  std::mutex m;
  std::vector<std::pair<char*, size_t>> r;
};
ArenaRegions& arena_regions() {
  static ArenaRegions* a = new ArenaRegions;
  return *a;
}
bool in_arena_region(void* p) {
  ArenaRegions& A = arena_regions();
  std::lock_guard<std::mutex> lk(A.m);
  for (auto& x : A.r)
    if (static_cast<char*>(p) >= x.first && static_cast<char*>(p) < x.first + x.second) return true;
  return false;
}
}  // namespace

void register_arena_region(void* base, size_t bytes) {
  ArenaRegions& A = arena_regions();
  std::lock_guard<std::mutex> lk(A.m);
  A.r.emplace_back(static_cast<char*>(base), bytes);
}

void* pool_alloc(size_t bytes) {
  if (g_arena) {
    const size_t start = (g_arena->used + 255) / 256 * 256;
    if (start + bytes > g_arena->cap)
      throw Error{TS_EINVAL, "problem does not fit in the " + std::to_string(g_arena->cap >> 20) +
                                 " MiB no-allocation scratch (a block of " + std::to_string(bytes) +
                                 " bytes after " + std::to_string(start) + " in use)"};
    g_arena->used = start + bytes;
    return g_arena->base + start;
  }
  int dev = 0;
  hip_check(hipGetDevice(&dev), "get device");
  const size_t sz = pool_round(bytes);
  Pool& P = pool();
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(P.m);
    DevicePool& D = P.dev[dev];
    auto it = D.free_blocks.lower_bound(sz);
    if (it != D.free_blocks.end() && it->first / 5 * 4 <= sz) {
      void* p = it->second;
      D.cached -= it->first;
      P.live[p] = {dev, it->first};
      D.free_blocks.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(P.m);
      DevicePool& D = P.dev[dev];
      for (auto& b : D.free_blocks) drop.push_back(b.second);
      D.free_blocks.clear();
      D.cached = 0;
    }
    for (void* b : drop) (void)hipFree(b);
    e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error{TS_ENOMEM, "hipMalloc of " + std::to_string(sz) + " bytes failed"};
    }
  }
  std::lock_guard<std::mutex> lk(P.m);
  P.live[p] = {dev, sz};
  return p;
}

void pool_release(void* p) {
  if (in_arena_region(p)) return;
  Pool& P = pool();
  bool free_now = std::uncaught_exceptions() > 0;
  {
    std::lock_guard<std::mutex> lk(P.m);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    const int dev = it->second.first;
    const size_t sz = it->second.second;
    P.live.erase(it);
    DevicePool& D = P.dev[dev];
    if (D.cap == 0) {
      size_t fr = 0, tot = 0;
      int cur = 0;
      (void)hipGetDevice(&cur);
      if (cur == dev && hipMemGetInfo(&fr, &tot) == hipSuccess) D.cap = std::min(size_t(8) << 30, tot / 16);
      else D.cap = size_t(1) << 30;
    }
    if (!free_now && D.cached + sz <= D.cap) {
      D.free_blocks.emplace(sz, p);
      D.cached += sz;
      return;
    }
  }
  (void)hipFree(p);
}

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory) throw Error{TS_ENOMEM, std::string(what) + ": out of device memory"};
  throw Error{TS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

// ---------------------------------------------------------------------------
// 1D Gram matrices of the cubic B-splines on [lo, hi] with N uniform
// intervals (Sec. 2.4): Psi_r[j, l] = int D^r B_j D^r B_l over the box.
// Each interval contributes the same 4x4 block (the four pieces alive there,
// as polynomials in t = (x - lo)/h - c), integrated exactly in t; the chain
// rule gives the factor h^(1 - 2r). Stored banded: band[j][o] = Psi[j][j+o-3].
static const double kPiece[4][4] = {
    // coefficients of t^0..t^3 of the pieces, times 6
    {1.0, -3.0, 3.0, -1.0},
    {4.0, 0.0, -6.0, 3.0},
    {1.0, 3.0, 3.0, -3.0},
    {0.0, 0.0, 0.0, 1.0},
};

static void piece_deriv(int a, int r, double out[4]) {
  double c[4];
  for (int i = 0; i < 4; ++i) c[i] = kPiece[a][i] / 6.0;
  for (int k = 0; k < r; ++k) {
    for (int i = 0; i < 3; ++i) c[i] = c[i + 1] * double(i + 1);
    c[3] = 0.0;
  }
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

void gram_band(double lo, double hi, int N, std::vector<double>& band /* [3][J][7] */) {
  const int J = N + kDeg;
  const double h = (hi - lo) / N;
  band.assign(size_t(3) * J * 7, 0.0);
  for (int r = 0; r < 3; ++r) {
    double loc[4][4];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        double pa[4], pb[4];
        piece_deriv(a, r, pa);
        piece_deriv(b, r, pb);
        double s = 0.0;
        for (int i = 0; i < 4; ++i)
          for (int j = 0; j < 4; ++j) s += pa[i] * pb[j] / double(i + j + 1);
        loc[a][b] = s * std::pow(h, 1.0 - 2.0 * r);
      }
    for (int c = 0; c < N; ++c)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) band[(size_t(r) * J + (c + a)) * 7 + (b - a + 3)] += loc[a][b];
  }
}

// u^e coefficient (e = 0..6) of b_a(u + 1/2) b_a'(u + 1/2), pair index a*4+a'.
void pair_table(std::vector<double>& ctab /* [7][16] */) {
  ctab.assign(7 * 16, 0.0);
  double shifted[4][4];
  for (int a = 0; a < 4; ++a) {
    for (int k = 0; k < 4; ++k) shifted[a][k] = 0.0;
    // t^i = (u + 1/2)^i = sum_k binom(i, k) u^k (1/2)^(i-k)
    for (int i = 0; i < 4; ++i) {
      const double ci = kPiece[a][i] / 6.0;
      double binom = 1.0;
      for (int k = 0; k <= i; ++k) {
        shifted[a][k] += ci * binom * std::pow(0.5, i - k);
        binom = binom * double(i - k) / double(k + 1);
      }
    }
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) ctab[(i + j) * 16 + a * 4 + b] += shifted[a][i] * shifted[b][j];
}

// Largest eigenvalue of the symmetric tridiagonal (alpha, beta) by bisection
// on the Sturm count.
double tridiag_max_eig(const std::vector<double>& al, const std::vector<double>& be) {
  const int m = int(al.size());
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(be[i]) : 0.0);
    lo = std::min(lo, al[i] - r);
    hi = std::max(hi, al[i] + r);
  }
  auto count_below = [&](double x) {  // eigenvalues < x
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
      const double b2 = (i > 0) ? be[i - 1] * be[i - 1] : 0.0;
      q = al[i] - x - (i > 0 ? b2 / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0.0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= m) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// ---------------------------------------------------------------------------
// Operator pieces.
template <typename T> static T* lvl_a(Level& L);
template <> double* lvl_a<double>(Level& L) { return L.a64.p; }
template <> float* lvl_a<float>(Level& L) { return L.a32.p; }
template <typename T> static T* lvl_b(Level& L);
template <> double* lvl_b<double>(Level& L) { return L.b64.p; }
template <> float* lvl_b<float>(Level& L) { return L.b32.p; }
template <typename T> static T* lvl_t(Level& L);
template <> double* lvl_t<double>(Level& L) { return L.t64.p; }
template <> float* lvl_t<float>(Level& L) { return L.t32.p; }
template <typename T> static const T* lvl_w(Level& L);
template <> const double* lvl_w<double>(Level& L) { return L.wdinv64.p; }
template <> const float* lvl_w<float>(Level& L) { return L.wdinv32.p; }
template <typename T> static const T* lvl_band(Level& L);
template <> const double* lvl_band<double>(Level& L) { return L.band64.p; }
template <> const float* lvl_band<float>(Level& L) { return L.band32.p; }
template <typename T> static T* prob_lamS(Problem* P);
template <> double* prob_lamS<double>(Problem* P) { return P->lamS64.p; }
template <> float* prob_lamS<float>(Problem* P) { return P->lamS32.p; }
template <typename T> static T* prob_xfer(Problem* P);
template <> double* prob_xfer<double>(Problem* P) { return P->xfer64.p; }
template <> float* prob_xfer<float>(Problem* P) { return P->xfer32.p; }

// out = lambda Lambda_g c by the three-accumulator recursion (Alg. 2): one
// kernel for d = 2, 3; for d >= 4 banded passes over the leading d - 3
// dimensions, then one kernel for the last three; one banded pass for d = 1.
template <typename T>
static void lambda_apply(Problem* P, int g, const T* c, T* out) {
  Level& L = P->lev[g];
  const int D = P->d;
  const int64_t K = L.K;
  if (D == 2 || D == 3) {
    hip_check(launch_lambda_fused<T>(D, c, out, lvl_band<T>(L), L.J, T(P->lam), P->stream), "lambda");
    return;
  }
  T* S = prob_lamS<T>(P);
  T* bufA = S;
  T* bufB = S + 3 * P->lev[P->G].K;
  const T* in0 = c;
  const T* in1 = nullptr;
  const T* in2 = nullptr;
  int64_t stride = K;
  if (D >= 4) {
    for (int p = 0; p < D - 3; ++p) {
      stride /= L.J;
      LambdaArgs<T> a{};
      a.in0 = in0; a.in1 = in1; a.in2 = in2;
      a.band = lvl_band<T>(L) + size_t(p) * 3 * L.J * 7;
      a.K = K; a.stride = stride; a.J = L.J;
      a.first = (p == 0); a.last = false;
      a.lam = T(P->lam);
      T* o = (p % 2 == 0) ? bufA : bufB;
      a.out0 = o; a.out1 = o + K; a.out2 = o + 2 * K;
      a.out = out;
      hip_check(launch_lambda_pass<T>(a, P->stream), "lambda pass");
      in0 = a.out0; in1 = a.out1; in2 = a.out2;
    }
    hip_check(launch_lambda_tail3<T>(in0, in1, in2, out, lvl_band<T>(L) + size_t(D - 3) * 3 * L.J * 7, L.J,
                                     K / (int64_t(L.J) * L.J * L.J), T(P->lam), P->stream),
              "lambda");
    return;
  }
  for (int p = 0; p < D; ++p) {
    stride /= L.J;
    LambdaArgs<T> a{};
    a.in0 = in0; a.in1 = in1; a.in2 = in2;
    a.band = lvl_band<T>(L) + size_t(p) * 3 * L.J * 7;
    a.K = K; a.stride = stride; a.J = L.J;
    a.first = (p == 0); a.last = (p == D - 1);
    a.lam = T(P->lam);
    T* o = (p % 2 == 0) ? bufA : bufB;
    a.out0 = o; a.out1 = o + K; a.out2 = o + 2 * K;
    a.out = out;
    hip_check(launch_lambda_pass<T>(a, P->stream), "lambda pass");
    in0 = a.out0; in1 = a.out1; in2 = a.out2;
  }
}

DataArgs data_args(Problem* P, int g, bool fp32, const void* c, void* out) {
  Level& L = P->lev[g];
  DataArgs a{};
  a.tfrac = fp32 ? static_cast<const void*>(P->t32.p) : static_cast<const void*>(P->t64.p);
  a.cell = P->cell.p;
  a.mkey = P->mkey.p;
  a.y = P->ys.p;
  a.off = P->off.p;
  a.c = c;
  a.out = out;
  a.n = P->n;
  a.G = P->G;
  a.g = g;
  a.tb = L.tb;
  a.ppb = P->ppb;
  if (L.wl_items.p) {
    a.wl_first = L.wl_first.p;
    a.wl_chunks = L.wl_chunks.p;
    a.wl_items = L.wl_items.p;
    a.wl_groups = L.wl_groups;
  }
  if (P->det) {
    a.det = 1;
    a.det_part = P->det_part.p;
    a.det_tile_first = L.det_tile_first.p;
  }
  return a;
}

// Work list of the point pass on level g, from the finest cell offsets
// (host copy `off`). The nonempty tiles, in Morton order, are cut into
// segments, segments into chunks of at most ppb points, chunks into items (a
// cell's run of at most Q points inside the chunk). Two ways of dealing
// segments to workgroups, chosen by what measured faster on MI355X:
// - split (d <= 3, small coefficient patches): workgroup w takes exactly the
//   points [w ppb, (w+1) ppb), so a tile that straddles a boundary becomes a
//   segment in each of the two workgroups;
// - packed (d >= 4, where staging and flushing a (2^tb+3)^d patch twice
//   costs more): whole tiles, cut only when longer than ppb, are packed into
//   workgroups of at most ppb points.
struct WorkListHost {
  std::vector<int32_t> first;   // per workgroup: its first chunk (one past the last entry: the end)
  std::vector<int4> chunks;
  std::vector<uint32_t> items;
  std::vector<int32_t> tile_first;   // per tile in Morton order: its first chunk; then the number of chunks
};

// Host side only (no device calls), so that it can run on a host thread.
static WorkListHost make_worklist(int D, int G, int g, int tb, int64_t ppb, const std::vector<int32_t>& off) {
  const bool split = D <= 3;
  const int sh = G - g;
  const int Q = kItemQ[D];
  const int64_t ch = ppb;
  const int cells_in_tile = 1 << (D * tb);
  const int64_t ntiles = int64_t(1) << (D * (g - tb));
  auto cell_start = [&](int64_t c) { return int64_t(off[size_t(c << (D * sh))]); };   // level-g Morton cell c
  WorkListHost w;
  std::vector<int32_t>& first = w.first;
  std::vector<int4>& chunks = w.chunks;
  std::vector<uint32_t>& items = w.items;
  int64_t wg_points = 0;
  w.tile_first.resize(size_t(ntiles) + 1);
  for (int64_t t = 0; t < ntiles; ++t) {
    w.tile_first[size_t(t)] = int32_t(chunks.size());   // the chunks of a tile are contiguous
    const int64_t c0 = t << (D * tb);
    const int64_t a = cell_start(c0), b = cell_start(c0 + cells_in_tile);
    if (a == b) continue;
    int j = 0;   // the first cell of the tile that still holds points at or after k0
    for (int64_t s0 = a, s1; s0 < b; s0 = s1) {
      // one segment [s0, s1) of the tile
      if (split) {
        s1 = std::min(b, (s0 / ch + 1) * ch);
        if (s0 % ch == 0) first.push_back(int32_t(chunks.size()));
      } else {
        s1 = std::min(b, s0 + ch);
        if (first.empty() || wg_points + (s1 - s0) > ch) {
          first.push_back(int32_t(chunks.size()));
          wg_points = 0;
        }
        wg_points += s1 - s0;
      }
      for (int64_t k0 = s0; k0 < s1; k0 += ch) {
        const int64_t k1 = std::min(s1, k0 + ch);
        uint32_t flags = uint32_t(t);
        if (k0 == s0) flags |= kChunkFirst;
        if (k1 == s1) flags |= kChunkLast;
        const size_t item0 = items.size();
        chunks.push_back(make_int4(int(k0), int(k1), int(item0), int(flags)));
        while (j < cells_in_tile && cell_start(c0 + j + 1) <= k0) ++j;
        for (int jj = j; jj < cells_in_tile; ++jj) {
          if (cell_start(c0 + jj) >= k1) break;
          const int64_t lo = std::max(cell_start(c0 + jj), k0), hi = std::min(cell_start(c0 + jj + 1), k1);
          for (int64_t q = lo; q < hi; q += Q)
            items.push_back(uint32_t(jj) | (uint32_t(q - k0) << kItemLoShift) |
                            (uint32_t(std::min<int64_t>(Q, hi - q)) << kItemCntShift));
        }
        // longest items first: the lane groups of a wave then get items of
        // similar length, and a wave runs as many steps as its longest item
        std::stable_sort(items.begin() + int64_t(item0), items.end(), [](uint32_t x, uint32_t y) {
          return (x >> kItemCntShift) > (y >> kItemCntShift);
        });
      }
    }
    if (int64_t(items.size()) >= INT32_MAX || int64_t(chunks.size()) >= INT32_MAX)
      throw Error{TS_EINVAL, "work list exceeds 2^31 entries"};
  }
  w.tile_first[size_t(ntiles)] = int32_t(chunks.size());
  first.push_back(int32_t(chunks.size()));
  chunks.push_back(make_int4(0, 0, int(items.size()), 0));
  if (items.empty()) items.push_back(0u);
  return w;
}

static void upload_worklist(Problem* P, int g, const WorkListHost& w) {
  Level& L = P->lev[g];
  const std::vector<int32_t>& first = w.first;
  const std::vector<int4>& chunks = w.chunks;
  const std::vector<uint32_t>& items = w.items;
  hipStream_t st = P->stream;
  L.wl_groups = int(first.size()) - 1;
  if (P->det) {
    // every chunk must be a whole segment: its patch is stored, not added
    for (size_t c = 0; c + 1 < chunks.size(); ++c)
      if ((uint32_t(chunks[c].w) & (kChunkFirst | kChunkLast)) != (kChunkFirst | kChunkLast))
        throw Error{TS_EINVAL, "work list chunk is not a whole segment"};
    L.det_tile_first.alloc(w.tile_first.size());
    hip_check(hipMemcpyAsync(L.det_tile_first.p, w.tile_first.data(), w.tile_first.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, st),
              "upload");
  }
  L.wl_first.alloc(first.size());
  L.wl_chunks.alloc(chunks.size());
  L.wl_items.alloc(items.size());
  hip_check(hipMemcpyAsync(L.wl_first.p, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice, st),
            "upload");
  hip_check(hipMemcpyAsync(L.wl_chunks.p, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice, st),
            "upload");
  hip_check(hipMemcpyAsync(L.wl_items.p, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st),
            "upload");
  hip_check(hipStreamSynchronize(st), "sync");   // host vectors go out of scope
}

template <typename T> static const T* lvl_S(Level& L);
template <> const double* lvl_S<double>(Level& L) { return L.S64.p; }
template <> const float* lvl_S<float>(Level& L) { return L.S32.p; }

// out = A_g c (Sec. 2.4): Lambda passes write out, the point pass adds
// Phi'Phi c; or, on a level assembled at setup, one stencil product.
template <typename T>
void apply_op(Problem* P, int g, const T* c, T* out) {
  if (P->general) {
    apply_general<T>(P, g, c, out);
    P->applies++;
    return;
  }
  Level& L = P->lev[g];
  if (L.stencil) {
    hip_check(launch_stencil_apply<T>(P->d, 0, lvl_S<T>(L), L.J, c, out, nullptr, nullptr, L.K, P->stream),
              "stencil apply");
    P->applies++;
    return;
  }
  lambda_apply<T>(P, g, c, out);
  const bool fp32 = sizeof(T) == 4;
  hip_check(launch_data(P->d, fp32, kApply, data_args(P, g, fp32, c, out), P->stream), "data pass");
  P->applies++;
}
template void apply_op<double>(Problem*, int, const double*, double*);
template void apply_op<float>(Problem*, int, const float*, float*);

// out (level g) = I e (level g-1), or out -= I e when subtract is set.
template <typename T>
void prolong_op(Problem* P, int g, const T* e, T* out, bool subtract) {
  if (P->general) {
    transfer_general<T>(P, g, true, e, out, static_cast<const T*>(nullptr), subtract);
    return;
  }
  const int D = P->d;
  const int Jc = P->lev[g - 1].J, Jf = P->lev[g].J;
  if (P->lev[g].K <= kFusedTransferMaxK) {
    hip_check(launch_transfer_fused<T>(D, true, e, nullptr, out, Jc, Jf, subtract ? 1 : 0, static_cast<const T*>(nullptr),
                                       static_cast<T*>(nullptr), P->stream),
              "prolongation");
    return;
  }
  T* X = prob_xfer<T>(P);
  T* bufs[2] = {X, X + P->lev[P->G].K};
  const T* in = e;
  for (int p = 0; p < D; ++p) {
    TransferArgs<T> a{};
    int64_t inner = 1;
    for (int q = p + 1; q < D; ++q) inner *= Jc;
    int64_t outer = 1;
    for (int q = 0; q < p; ++q) outer *= Jf;
    a.in = in;
    a.out = (p == D - 1) ? out : bufs[p % 2];
    a.Kout = outer * Jf * inner;
    a.inner = inner;
    a.Jc = Jc; a.Jf = Jf;
    a.subtract = (p == D - 1 && subtract) ? 1 : 0;
    hip_check(launch_transfer<T>(true, a, P->stream), "prolongation pass");
    in = a.out;
  }
}
template void prolong_op<double>(Problem*, int, const double*, double*, bool);
template void prolong_op<float>(Problem*, int, const float*, float*, bool);

// out (level g-1) = I' (r - sub) (level g); sub may be null. With a0 set
// (cubic form only) also a0 = w0 .* out, the first Jacobi sweep from zero of
// level g-1.
template <typename T>
void restrict_op(Problem* P, int g, const T* r, T* out, const T* sub, const T* w0, T* a0) {
  if (P->general) {
    transfer_general<T>(P, g, false, r, out, sub, false);
    return;
  }
  const int D = P->d;
  const int Jc = P->lev[g - 1].J, Jf = P->lev[g].J;
  if (P->lev[g].K <= kFusedTransferMaxK && D <= 4) {   // (d = 5 would keep its gather tables in scratch)
    hip_check(launch_transfer_fused<T>(D, false, r, sub, out, Jc, Jf, 0, w0, a0, P->stream), "restriction");
    return;
  }
  T* X = prob_xfer<T>(P);
  T* bufs[2] = {X, X + P->lev[P->G].K};
  const T* in = r;
  for (int p = 0; p < D; ++p) {
    TransferArgs<T> a{};
    int64_t inner = 1;
    for (int q = p + 1; q < D; ++q) inner *= Jf;
    int64_t outer = 1;
    for (int q = 0; q < p; ++q) outer *= Jc;
    a.in = in;
    a.out = (p == D - 1) ? out : bufs[p % 2];
    a.Kout = outer * Jc * inner;
    a.inner = inner;
    a.Jc = Jc; a.Jf = Jf;
    a.subtract = 0;
    a.sub = (p == 0) ? sub : nullptr;
    a.w = (p == D - 1) ? w0 : nullptr;
    a.a = (p == D - 1) ? a0 : nullptr;
    hip_check(launch_transfer<T>(false, a, P->stream), "restriction pass");
    in = a.out;
  }
}
template void restrict_op<double>(Problem*, int, const double*, double*, const double*, const double*, double*);
template void restrict_op<float>(Problem*, int, const float*, float*, const float*, const float*, float*);

// Coarse CG slots (the outer Krylov loop uses 0..7, Lanczos 16..).
enum CoarseSlot : int { kCbb = 8, kCrzA = 9, kCrzB = 10, kCpv = 11, kCrr = 12 };

// x = A_c^-1 b on the coarsest level c (Sec. 3.2.4).
// Direct: the precomputed inverse B and one refinement step, x1 = B b,
// r = b - A_c x1, x = x1 + B r (all FP64), as accurate as a backward-stable
// solve. CG: matrix-free CG on A_c with D_c^-1 as preconditioner from x = 0,
// in FP64, until ||r|| <= coarse_tol ||b|| or coarse_max_iter iterations; the
// residual norm is read back every few iterations.
template <typename T>
void coarse_op(Problem* P, const T* b, T* x) {
  const int K = P->K1;
  if (P->opt.coarse_solver != TS_COARSE_CG) {
    double* x1 = P->cwork.p;
    double* r = P->cwork.p + K;
    hip_check(launch_gemv<double, T, double>(P->A1inv.p, K, nullptr, 1.0, b, x1, P->stream), "coarse solve");
    hip_check(launch_gemv<T, double, double>(P->A1.p, K, b, -1.0, x1, r, P->stream), "coarse residual");
    hip_check(launch_gemv<double, double, T>(P->A1inv.p, K, x1, 1.0, r, x, P->stream), "coarse correction");
    return;
  }
  hipStream_t st = P->stream;
  const int c = P->Gc;
  double *cx = P->cx.p, *cr = P->cr.p, *cz = P->cz.p, *cp = P->cp.p, *cv = P->cv.p;
  hip_check(launch_scale_copy<T, double>(b, cr, K, 1.0, nullptr, st), "coarse copy");
  hip_check(launch_fill<double>(cx, 0.0, K, st), "fill");
  dot_op<double, double>(P, cr, cr, K, kCbb);
  hip_check(launch_mul(P->cdinv.p, cr, cz, K, st), "coarse precondition");
  hip_check(launch_scale_copy<double, double>(cz, cp, K, 1.0, nullptr, st), "copy");
  int sa = kCrzA, sb = kCrzB;
  dot_op<double, double>(P, cr, cz, K, sa);
  const double tol = P->opt.coarse_tol > 0.0 ? P->opt.coarse_tol : 1e-14;
  const int maxit = P->opt.coarse_max_iter > 0 ? P->opt.coarse_max_iter : 20000;
  constexpr int kCheck = 8;
  for (int it = 0; it < maxit;) {
    for (int j = 0; j < kCheck && it < maxit; ++j, ++it) {
      apply_op<double>(P, c, cp, cv);
      dot_op<double, double>(P, cp, cv, K, kCpv);
      hip_check(launch_cg_step<double, double>(cx, cr, cp, cv, K, P->slot(sa), P->slot(kCpv), st), "coarse step");
      hip_check(launch_mul(P->cdinv.p, cr, cz, K, st), "coarse precondition");
      dot_op<double, double>(P, cr, cz, K, sb);
      hip_check(launch_p_update<double>(cp, cz, K, P->slot(sb), P->slot(sa), st), "coarse p update");
      std::swap(sa, sb);
      ++P->coarse_iters;
    }
    dot_op<double, double>(P, cr, cr, K, kCrr);
    double h[5];
    P->read_slots(kCbb, 5, h);
    const double bb = h[0], rr = h[kCrr - kCbb];
    if (!(bb > 0.0) || !(rr > tol * tol * bb)) break;
  }
  hip_check(launch_scale_copy<double, T>(cx, x, K, 1.0, nullptr, st), "coarse copy");
}
template void coarse_op<double>(Problem*, const double*, double*);
template void coarse_op<float>(Problem*, const float*, float*);

// One symmetric SSOR step on a stencil level (Sec. 3.2.2): the 4^d colour
// classes forward, then backward; each class update is
// x_k += omega (b_k - (A x)_k) / A_kk for every row k of the class at once.
template <typename T>
static void ssor_step(Problem* P, int g, T* x, const T* b) {
  Level& L = P->lev[g];
  int ncol = 1;
  for (int p = 0; p < P->d; ++p) ncol *= 4;
  const T w = T(P->opt.ssor_omega);
  for (int c = 0; c < ncol; ++c)
    hip_check(launch_stencil_color<T>(P->d, lvl_S<T>(L), L.J, x, b, w, c, L.K, P->stream), "ssor");
  for (int c = ncol - 1; c >= 0; --c)
    hip_check(launch_stencil_color<T>(P->d, lvl_S<T>(L), L.J, x, b, w, c, L.K, P->stream), "ssor");
  P->applies += 2;
}

int bottom_level(const Problem* P) {
  if (P->bottom_g == 0 || P->opt.smoother != TS_SMOOTH_JACOBI || P->opt.coarse_solver != TS_COARSE_DIRECT ||
      P->opt.nu1 != P->bottom_nu1 || P->opt.nu2 != P->bottom_nu2)
    return 0;
  return P->bottom_g;
}

template <typename T> static const T* bottom_op(Problem* P);
template <> const double* bottom_op<double>(Problem* P) { return P->bottom64.p; }
template <> const float* bottom_op<float>(Problem* P) { return P->bottom32.p; }

// Where the first Jacobi sweep of the V-cycle on level g (g below the finest)
// lands, when that sweep is the plain product alpha = w .* b that the
// restriction producing b can write as well; null when it is not (coarsest
// level, no pre-smoothing, SSOR, a stencil level whose first two sweeps are
// one fused product, the general form).
// (alpha: the output of that V-cycle.)
template <typename T>
T* first_sweep_target(Problem* P, int g, T* alpha) {
  if (P->general || g <= P->Gc || P->opt.nu1 < 1 || g == bottom_level(P)) return nullptr;
  Level& L = P->lev[g];
  if (L.stencil) {
    if (P->opt.smoother == TS_SMOOTH_SSOR || P->opt.nu1 != 1) return nullptr;
    // the stencil branch below ping-pongs nu2 times after the first sweep
    return (P->opt.nu2 % 2 == 0) ? alpha : lvl_t<T>(L);
  }
  return alpha;
}
template double* first_sweep_target<double>(Problem*, int, double*);
template float* first_sweep_target<float>(Problem*, int, float*);

template <typename T>
static T* first_sweep_dest(Problem* P, int g) {
  return first_sweep_target<T>(P, g, lvl_a<T>(P->lev[g]));
}

// The next coarser level's recursion: restriction of r (minus sub) to b_{g-1},
// with the first sweep of level g-1 fused into it where possible, then the
// V-cycle on level g-1.
template <typename T>
static void descend(Problem* P, int g, const T* r, const T* sub) {
  Level& C = P->lev[g - 1];
  T* a0 = first_sweep_dest<T>(P, g - 1);
  restrict_op<T>(P, g, r, lvl_b<T>(C), sub, a0 ? lvl_w<T>(C) : static_cast<const T*>(nullptr), a0);
  vcycle_op<T>(P, g - 1, lvl_b<T>(C), lvl_a<T>(C), a0 != nullptr);
}

// One V-cycle (Alg. 7) on level g from a zero start: alpha = B_g b.
template <typename T>
void vcycle_op(Problem* P, int g, const T* b, T* alpha, bool pre_done) {
  if (g == P->Gc) {
    coarse_op<T>(P, b, alpha);
    return;
  }
  if (g == bottom_level(P)) {   // the whole V-cycle from here down: alpha = B_g b
    hip_check(launch_bottom_gemv<T, T>(bottom_op<T>(P), int(P->lev[g].K), b, alpha, P->stream), "bottom");
    return;
  }
  Level& L = P->lev[g];
  Level& C = P->lev[g - 1];
  const int64_t K = L.K;
  T* t = lvl_t<T>(L);
  const T* w = lvl_w<T>(L);
  const int nu1 = P->opt.nu1, nu2 = P->opt.nu2;
  if (L.stencil && P->opt.smoother == TS_SMOOTH_SSOR) {
    // SSOR steps in place on alpha; the residual through the stencil product
    hip_check(launch_fill<T>(alpha, T(0), K, P->stream), "fill");
    for (int j = 0; j < nu1; ++j) ssor_step<T>(P, g, alpha, b);
    hip_check(launch_stencil_apply<T>(P->d, 2, lvl_S<T>(L), L.J, alpha, t, b, w, K, P->stream), "residual");
    P->applies++;
    descend<T>(P, g, t, static_cast<const T*>(nullptr));
    prolong_op<T>(P, g, lvl_a<T>(C), alpha, true);
    for (int j = 0; j < nu2; ++j) ssor_step<T>(P, g, alpha, b);
    return;
  }
  if (L.stencil) {
    // Jacobi sweeps fused into the stencil product, ping-ponging between
    // alpha and t; the first sweep lands so that the last one ends in alpha.
    // (the first two sweeps from zero are one fused product)
    const T* S = lvl_S<T>(L);
    const int swaps = std::max(0, nu1 - 2) + nu2;
    T* cur = (swaps % 2 == 0) ? alpha : t;
    T* oth = (cur == alpha) ? t : alpha;
    if (nu1 >= 2) {
      hip_check(launch_stencil_apply<T>(P->d, 3, S, L.J, nullptr, cur, b, w, K, P->stream), "jacobi");
      P->applies++;
      for (int j = 2; j < nu1; ++j) {
        hip_check(launch_stencil_apply<T>(P->d, 1, S, L.J, cur, oth, b, w, K, P->stream), "jacobi");
        P->applies++;
        std::swap(cur, oth);
      }
    } else if (nu1 == 1) {
      if (!pre_done) hip_check(launch_jacobi_first<T>(cur, w, b, K, P->stream), "jacobi");
    } else {
      hip_check(launch_fill<T>(cur, T(0), K, P->stream), "fill");
    }
    hip_check(launch_stencil_apply<T>(P->d, 2, S, L.J, cur, oth, b, w, K, P->stream), "residual");
    P->applies++;
    descend<T>(P, g, oth, static_cast<const T*>(nullptr));
    prolong_op<T>(P, g, lvl_a<T>(C), cur, true);
    for (int j = 0; j < nu2; ++j) {
      hip_check(launch_stencil_apply<T>(P->d, 1, S, L.J, cur, oth, b, w, K, P->stream), "jacobi");
      P->applies++;
      std::swap(cur, oth);
    }
    if (cur != alpha)
      hip_check(launch_scale_copy<T, T>(cur, alpha, K, 1.0, nullptr, P->stream), "copy");
    return;
  }
  // pre-smoothing (Alg. 6); the first sweep from zero needs no apply
  if (nu1 >= 1) {
    if (!pre_done) hip_check(launch_jacobi_first<T>(alpha, w, b, K, P->stream), "jacobi");
    for (int j = 1; j < nu1; ++j) {
      apply_op<T>(P, g, alpha, t);
      hip_check(launch_jacobi<T>(alpha, w, b, t, K, P->stream), "jacobi");
    }
  } else {
    hip_check(launch_fill<T>(alpha, T(0), K, P->stream), "fill");
  }
  // r = A alpha - b, restricted (the subtraction is fused into the restriction)
  apply_op<T>(P, g, alpha, t);
  descend<T>(P, g, static_cast<const T*>(t), b);
  // alpha -= I e
  prolong_op<T>(P, g, lvl_a<T>(C), alpha, true);
  // post-smoothing
  for (int j = 0; j < nu2; ++j) {
    apply_op<T>(P, g, alpha, t);
    hip_check(launch_jacobi<T>(alpha, w, b, t, K, P->stream), "jacobi");
  }
}
template void vcycle_op<double>(Problem*, int, const double*, double*, bool);
template void vcycle_op<float>(Problem*, int, const float*, float*, bool);

// Times `reps` launches of the Lambda passes and of the point pass of A_g.
template <typename T>
void profile_apply(Problem* P, int g, int reps, double* ms_lambda, double* ms_data) {
  Level& L = P->lev[g];
  T* c = lvl_a<T>(L);
  T* out = lvl_t<T>(L);
  hip_check(launch_fill<T>(c, T(0.5), L.K, P->stream), "fill");
  hipEvent_t e0, e1, e2;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  hip_check(hipEventCreate(&e2), "event");
  const bool fp32 = sizeof(T) == 4;
  const DataArgs a = data_args(P, g, fp32, c, out);
  if (P->general) {
    profile_general<T>(P, g, c, out, reps, e0, e1, e2);
  } else {
  hip_check(hipEventRecord(e0, P->stream), "record");
  for (int i = 0; i < reps; ++i) lambda_apply<T>(P, g, c, out);
  hip_check(hipEventRecord(e1, P->stream), "record");
  for (int i = 0; i < reps; ++i) hip_check(launch_data(P->d, fp32, kApply, a, P->stream), "data pass");
  hip_check(hipEventRecord(e2, P->stream), "record");
  }
  hip_check(hipEventSynchronize(e2), "sync");
  float t01 = 0.f, t12 = 0.f;
  hip_check(hipEventElapsedTime(&t01, e0, e1), "elapsed");
  hip_check(hipEventElapsedTime(&t12, e1, e2), "elapsed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);
  *ms_lambda = double(t01) / reps;
  *ms_data = double(t12) / reps;
}
template void profile_apply<double>(Problem*, int, int, double*, double*);
template void profile_apply<float>(Problem*, int, int, double*, double*);

// ---------------------------------------------------------------------------
// Device scalars: dots go to slots; read back with one synchronising copy.
double* Problem::slot(int i) { return slots.p + i; }

void Problem::copy_slots(int first, int count) {
  hip_check(hipMemcpyAsync(host_slots + first, slots.p + first, sizeof(double) * count, hipMemcpyDeviceToHost,
                           stream),
            "slot readback");
  if (slots_ready) hip_check(hipEventRecord(slots_ready, stream), "record");
}

void Problem::wait_slots(int first, int count, double* host) {
  if (slots_ready) hip_check(hipEventSynchronize(slots_ready), "event sync");
  else hip_check(hipStreamSynchronize(stream), "stream sync");
  std::memcpy(host, host_slots + first, sizeof(double) * count);
}

void Problem::read_slots(int first, int count, double* host) {
  hip_check(hipMemcpyAsync(host_slots + first, slots.p + first, sizeof(double) * count, hipMemcpyDeviceToHost,
                           stream),
            "slot readback");
  hip_check(hipStreamSynchronize(stream), "stream sync");
  std::memcpy(host, host_slots + first, sizeof(double) * count);
}

template <typename TX, typename TY>
void dot_op(Problem* P, const TX* x, const TY* y, int64_t K, int slot) {
  hip_check(launch_dot<TX, TY>(x, y, K, P->partial.p, P->slot(slot), P->stream), "dot");
}
template void dot_op<double, double>(Problem*, const double*, const double*, int64_t, int);
template void dot_op<float, float>(Problem*, const float*, const float*, int64_t, int);

// ---------------------------------------------------------------------------
// Setup.

static void compute_diag(Problem* P, int g) {
  if (P->general) {
    diag_general(P, g);
    return;
  }
  Level& L = P->lev[g];
  hip_check(launch_lambda_diag(P->d, L.band64.p, L.J, L.K, P->lam, L.diag.p, P->stream), "lambda diag");
  hip_check(launch_data(P->d, false, kDiag, data_args(P, g, false, nullptr, L.diag.p), P->stream), "data diag");
}

// theta_g: largest Ritz value of `steps` Lanczos steps on D^-1/2 A_g D^-1/2
// from the fixed start u[k] = frac(k * 2654435761 / 2^32) - 1/2.
// The Lanczos scalars stay on the device (each step's kernels read the
// previous ones from slots); the host reads them once per batch of steps and
// applies the early stop afterwards (steps past it are discarded).
static double lanczos_theta(Problem* P, int g, int steps) {
  Level& L = P->lev[g];
  const int64_t K = L.K;
  double* dis = P->vb.p;   // PCG vectors double as work space during setup
  double* v = P->vr.p;
  double* vprev = P->vz.p;
  double* w = P->vp.p;
  double* y = P->vv.p;
  double* Ay = L.t64.p;
  constexpr int kBatch = (kSlots - kLanczosSlot0 - 1) / 2;
  hip_check(launch_rsqrt_vec(L.diag.p, dis, K, P->stream), "rsqrt");
  hip_check(launch_start_vector(w, K, P->stream), "start");
  dot_op<double, double>(P, w, w, K, kLanczosSlot0);
  hip_check(launch_scale_copy<double, double>(w, v, K, 1.0, P->slot(kLanczosSlot0), P->stream), "scale");
  hip_check(launch_fill<double>(vprev, 0.0, K, P->stream), "fill");
  std::vector<double> al, be, h(size_t(2) * kBatch);
  const int m = int(std::min<int64_t>(steps, K));
  const double* b2prev = nullptr;
  bool done = false;
  for (int j = 0; j < m && !done;) {
    const int nb = std::min(kBatch, m - j);
    for (int i = 0; i < nb; ++i) {
      const int sa = kLanczosSlot0 + 1 + 2 * i, sb = sa + 1;
      hip_check(launch_mul(dis, v, y, K, P->stream), "mul");
      apply_op<double>(P, g, y, Ay);
      hip_check(launch_lanczos_w(dis, Ay, vprev, b2prev, w, K, P->stream), "lanczos");
      dot_op<double, double>(P, w, v, K, sa);                                       // a
      hip_check(launch_axpy(-1.0, P->slot(sa), v, w, K, P->stream), "axpy");     // w -= a v
      dot_op<double, double>(P, w, w, K, sb);                                       // b^2
      std::swap(vprev, v);   // vprev <- v
      hip_check(launch_scale_copy<double, double>(w, v, K, 1.0, P->slot(sb), P->stream), "scale");
      b2prev = P->slot(sb);
    }
    P->read_slots(kLanczosSlot0 + 1, 2 * nb, h.data());
    for (int i = 0; i < nb; ++i, ++j) {
      const double a = h[size_t(2 * i)], b = std::sqrt(h[size_t(2 * i + 1)]);
      al.push_back(a);
      if (j == m - 1 || b <= 1e-12 * std::fabs(a)) {
        done = true;
        break;
      }
      be.push_back(b);
    }
  }
  be.resize(al.size() > 0 ? al.size() - 1 : 0);
  return tridiag_max_eig(al, be);
}

// Assembles A_g of level g as a 7^d-point stencil: level moments, d
// Kronecker passes with the pair table, then lambda Lambda_g and the
// offset-major layout.
// mom: on entry the moments of level g if the caller has them (from the level
// above), else empty; on return the moments of level g-1 if want_coarser.
static void build_stencil(Problem* P, int g, DevBuf<double>& mom, bool want_coarser) {
  Level& L = P->lev[g];
  const int D = P->d, N = L.N, J = L.J;
  int64_t NO = 1, in_sz = 1, max_sz = 0;
  for (int p = 0; p < D; ++p) { NO *= 7; in_sz *= int64_t(7) * N; }
  max_sz = in_sz;
  {
    int64_t sz = in_sz;
    for (int p = 0; p < D; ++p) { sz = sz / (int64_t(7) * N) * (int64_t(7) * J); max_sz = std::max(max_sz, sz); }
  }
  DevBuf<double> bufA, bufB, ctab, coarser;
  std::vector<double> ct;
  pair_table(ct);
  ctab.alloc(ct.size());
  hip_check(hipMemcpyAsync(ctab.p, ct.data(), ct.size() * sizeof(double), hipMemcpyHostToDevice, P->stream),
            "upload");
  const double* src = mom.p;
  if (!src) {
    bufA.alloc(size_t(max_sz));
    hip_check(launch_fill<double>(bufA.p, 0.0, in_sz, P->stream), "fill");
    hip_check(launch_level_moments(D, P->t64.p, P->cell.p, P->off.p, P->n, P->G, g, bufA.p, P->det, P->stream),
              "moments");
    src = bufA.p;
  }
  bufB.alloc(size_t(max_sz));
  if (want_coarser && g > 1) {
    // level g-1 moments, one dimension at a time through two regions of bufB
    // (each pass halves the size)
    const int Nc = N / 2;
    int64_t csz = 1;
    for (int p = 0; p < D; ++p) csz *= int64_t(7) * Nc;
    coarser.alloc(size_t(csz));
    double* region[2] = {bufB.p, bufB.p + in_sz / 2};
    const double* cin = src;
    for (int p = 0; p < D; ++p) {
      int64_t outer = 1, inner = 1;
      for (int q = 0; q < p; ++q) outer *= int64_t(7) * Nc;
      for (int q = p + 1; q < D; ++q) inner *= int64_t(7) * N;
      double* cout = (p == D - 1) ? coarser.p : region[p % 2];
      hip_check(launch_moments_coarsen(cin, cout, Nc, outer, inner, P->stream), "coarsen moments");
      cin = cout;
    }
  }
  double* cur = bufA.p;
  double* nxt = bufB.p;
  for (int p = 0; p < D; ++p) {
    int64_t outer = 1, inner = 1;
    for (int q = 0; q < p; ++q) outer *= int64_t(7) * J;
    for (int q = p + 1; q < D; ++q) inner *= int64_t(7) * N;
    hip_check(launch_stencil_pass(p == 0 ? src : cur, nxt, ctab.p, N, outer, inner, P->stream), "stencil pass");
    if (p == 0 && !bufA.p) {   // the moments came from the caller: trade them for the second buffer
      hip_check(hipStreamSynchronize(P->stream), "sync");
      mom.reset();
      bufA.alloc(size_t(max_sz));
      cur = bufA.p;
    }
    std::swap(cur, nxt);
  }
  const int64_t NH = (NO + 1) / 2;   // stored half of the offsets (A_g is symmetric)
  L.S64.alloc(size_t(NH * L.K));
  L.S32.alloc(size_t(NH * L.K));
  hip_check(launch_stencil_finalize(D, cur, L.band64.p, J, L.K, P->lam, L.S64.p, L.S32.p, P->stream), "finalize");
  hip_check(hipStreamSynchronize(P->stream), "sync");   // temporaries and host tables go out of scope
  mom = std::move(coarser);
  L.stencil = true;
}

// Which levels get an assembled stencil: it must fit the memory budget and,
// in automatic mode, its estimated time (a stream of 8 bytes per entry at
// about 5 TB/s) must beat the point pass (about 0.5 ps per point and patch
// entry, as measured for the FP64 point pass on MI355X).
static bool want_stencil(int d, int J, int64_t n, int mode, double budget) {
  if (mode == 1) return false;
  double NO = 1.0, P4 = 1.0, K = 1.0, transient = 1.0;
  for (int p = 0; p < d; ++p) { NO *= 7.0; P4 *= 4.0; K *= J; transient *= 7.0 * J; }
  const double entries = NO * K;
  const double bytes = (NO + 1.0) / 2.0 * K * 12.0 + 2.0 * transient * 8.0;   // the stored half, FP64 + FP32
  if (bytes > budget) return false;
  if (mode == 2) return true;
  return entries * 1.6e-12 < double(n) * P4 * 0.5e-12;
}

// Largest level size whose V-cycle operator is assembled when bottom_max_k
// is 0: in the cubic form, where the levels it replaces are stencil products
// of a few microseconds each; in the general form, where each of them
// streams all n points, up to a larger size.
constexpr int64_t kBottomMaxK = 2744;
constexpr int64_t kBottomMaxKGeneral = 6000;

// The level from which the V-cycle is assembled as one dense operator, for
// these options and level sizes (0: none): the largest g below the finest,
// above the coarsest, with every level from c + 1 to g assemblable (held as
// a stencil in the cubic form; from the points in the general form) and K_g
// within the cap.
int choose_bottom(const ts_options& o, int Gc, int G, const std::vector<int64_t>& K, const std::vector<char>& ok,
                  bool general) {
  if (o.bottom_max_k < 0 || o.coarse_solver == TS_COARSE_CG || o.smoother != TS_SMOOTH_JACOBI ||
      o.preconditioner != TS_PC_MG)
    return 0;
  const int64_t cap = o.bottom_max_k > 0 ? o.bottom_max_k : (general ? kBottomMaxKGeneral : kBottomMaxK);
  int gb = 0;
  for (int g = Gc + 1; g < G; ++g) {
    if (K[size_t(g)] > cap || !ok[size_t(g)]) break;
    gb = g;
  }
  return gb;
}

static double stencil_budget_for(double stencil_budget) {
  if (stencil_budget > 0.0) return stencil_budget;
  if (g_arena) return 0.5 * double(g_arena->cap - std::min(g_arena->cap, g_arena->used));
  size_t free_b = 0, total_b = 0;
  hip_check(hipMemGetInfo(&free_b, &total_b), "meminfo");
  return std::min(16e9, 0.4 * double(free_b));
}

int64_t footprint_bytes(int d, int N, int64_t n, const ts_options& opt, double stencil_budget) {
  int G = 0;
  while ((1 << G) < N) ++G;
  auto ipow = [](int64_t b, int e) { int64_t r = 1; for (int i = 0; i < e; ++i) r *= b; return r; };
  const int64_t KG = ipow(N + kDeg, d);
  const int64_t cells = int64_t(1) << (G * d);
  // points: t64, t32, C-order cell, Morton key, responses; cell offsets
  const int64_t points = n * (12 * int64_t(d) + 16) + 4 * (cells + 1);
  // binning and sort temporaries (keys and indices double-buffered, radix
  // sort scratch bounded by another key/value pair and 1 MB)
  const int64_t sort_tmp = 24 * n + (1 << 20);
  int64_t levels = 0, stencils = 0, stencil_tmp = 0, det_part = 0;
  const int Gc = std::max(1, std::min(G, opt.coarsest_level));
  const bool direct = opt.coarse_solver != TS_COARSE_CG;
  const bool det = opt.deterministic == 1;
  std::vector<int64_t> Kl(size_t(G) + 1, 0);
  std::vector<char> stl(size_t(G) + 1, 0);
  for (int g = Gc; g <= G; ++g) {
    const int J = (1 << g) + kDeg;
    const int64_t K = ipow(J, d);
    levels += 56 * K + int64_t(d) * 3 * J * 7 * 12;
    const bool st = want_stencil(d, J, n, opt.stencil_mode, stencil_budget_for(stencil_budget));
    Kl[size_t(g)] = K;
    stl[size_t(g)] = st;
    if (!st || det) {   // work list: items <= n; workgroups <= chunks <= nonempty tiles
                        // + n / 64 (ppb >= 64)
      const int tb = std::min(kTileBits[d], g);
      const int64_t ntiles = int64_t(1) << (d * (g - tb));
      const int64_t chunks = std::min(n, ntiles) + n / 64 + 2;
      levels += 20 * chunks + 4 * n + 4;
      if (det) {   // the tile index and the stored patches of the largest level
        levels += 4 * (ntiles + 1);
        det_part = std::max(det_part, chunks * ipow((int64_t(1) << tb) + kDeg, d) * 8);
      }
    }
    // with the direct coarse solver level c carries its stencil: A_c is expanded from it
    if ((g == Gc && direct) || st) {
      stencils += (ipow(7, d) + 1) / 2 * K * 12;   // the stored half, FP64 + FP32
      // two pass buffers, plus the moments handed on to level g-1
      const int64_t coarser = g > 1 ? ipow(7 * int64_t(1 << (g - 1)), d) * 8 : 0;
      stencil_tmp = std::max(stencil_tmp, 2 * ipow(7 * int64_t(J), d) * 8 + coarser + (1 << 16));
    }
  }
  const int64_t K1 = ipow((int64_t(1) << Gc) + kDeg, d);
  const int64_t coarse = direct ? 2 * K1 * K1 * 8 + 2 * K1 * 8 : 6 * K1 * 8 + K1 * 4;
  // the dense V-cycle operator (FP64 + FP32) and, while it is assembled,
  // five K_g x K_g and four K_{g-1} x K_g matrices and B_{g-1}
  int64_t bottom = 0, bottom_tmp = 0;
  {
    const int gb = choose_bottom(opt, Gc, G, Kl, stl, false);
    for (int g = Gc + 1; g <= gb; ++g) {
      const int64_t Kf = Kl[size_t(g)], Kc = Kl[size_t(g) - 1];
      bottom_tmp = std::max(bottom_tmp, (5 * Kf * Kf + 4 * Kc * Kf + Kc * Kc) * 8);
    }
    if (gb > 0) bottom = Kl[size_t(gb)] * Kl[size_t(gb)] * 12;
  }
  const int64_t finest = KG * (6 * 12 + 2 * 12 + 5 * 8 + 5 * 4);
  const int64_t misc = 16 * 8 + 3 * kMaxPartials * 8 + 64;
  const int64_t steady = points + levels + stencils + coarse + finest + misc + det_part + bottom;
  // allocation granularity: round every buffer up, roughly 40 buffers per level
  const int64_t slack = int64_t(64) * 4096 * (G + 2);
  return steady + std::max({sort_tmp, stencil_tmp, bottom_tmp}) + slack;
}

// The coarse solver of level c (Sec. 3.2.4). Direct: A_c expanded from the
// level-c stencil (built here if the apply path did not build it), then
// inverted by Gauss-Jordan; pivots checked for positivity. CG: the inverse
// diagonal and the CG vectors of level c.
static void build_coarse(Problem* P) {
  const int D = P->d;
  const int c = P->Gc;
  Level& L1 = P->lev[c];
  const int64_t K1 = L1.K;
  P->K1 = int(K1);
  if (P->opt.coarse_solver == TS_COARSE_CG) {
    P->cdinv.alloc(size_t(K1));
    P->cx.alloc(size_t(K1));
    P->cr.alloc(size_t(K1));
    P->cz.alloc(size_t(K1));
    P->cp.alloc(size_t(K1));
    P->cv.alloc(size_t(K1));
    DevBuf<float> unused;
    unused.alloc(size_t(K1));
    hip_check(launch_wdinv(L1.diag.p, 1.0, P->cdinv.p, unused.p, K1, P->stream), "coarse dinv");
    hip_check(hipStreamSynchronize(P->stream), "sync");
    return;
  }
  if (!P->general && !L1.S64.p) {
    DevBuf<double> none;
    build_stencil(P, c, none, false);
    L1.stencil = (P->opt.stencil_mode != 1);
  }
  DevBuf<double> row, col, piv;
  P->A1.alloc(size_t(K1) * K1);
  P->A1inv.alloc(size_t(K1) * K1);
  P->cwork.alloc(size_t(2 * K1));
  if (P->general) {
    coarse_matrix_general(P, P->A1.p);
  } else {
    hip_check(launch_fill<double>(P->A1.p, 0.0, K1 * K1, P->stream), "fill");
    hip_check(launch_dense_from_stencil(D, L1.S64.p, L1.J, K1, P->A1.p, P->stream), "assemble");
  }
  // A_c^-1 = S (S A_c S)^-1 S with S = diag(A_c)^-1/2: the Jacobi-scaled
  // matrix, whose condition number is far smaller where a few B-splines
  // carry little data, is inverted (its explicit inverse is then accurate
  // in the energy norm of A_c, which the V-cycle sees)
  DevBuf<double> sc;
  sc.alloc(size_t(K1));
  hip_check(hipMemcpyAsync(P->A1inv.p, P->A1.p, sizeof(double) * K1 * K1, hipMemcpyDeviceToDevice, P->stream),
            "copy A1");
  hip_check(launch_inv_sqrt_diag(P->A1.p, int(K1), sc.p, P->stream), "coarse scaling");
  hip_check(launch_sym_scale(P->A1inv.p, int(K1), sc.p, P->stream), "coarse scaling");
  row.alloc(size_t(K1));
  col.alloc(size_t(K1));
  piv.alloc(size_t(K1));
  for (int k = 0; k < K1; ++k)
    hip_check(launch_gj_step(P->A1inv.p, int(K1), k, row.p, col.p, piv.p, P->stream), "gauss-jordan");
  hip_check(launch_sym_scale(P->A1inv.p, int(K1), sc.p, P->stream), "coarse scaling");
  hip_check(launch_symmetrize(P->A1inv.p, int(K1), P->stream), "symmetrize");
  std::vector<double> pv(static_cast<size_t>(K1));
  hip_check(hipMemcpyAsync(pv.data(), piv.p, pv.size() * sizeof(double), hipMemcpyDeviceToHost, P->stream),
            "download");
  hip_check(hipStreamSynchronize(P->stream), "sync");
  // pivots of the scaled matrix (unit diagonal): pivot_k / A_kk of the original
  for (int64_t k = 0; k < K1; ++k) {
    if (!std::isfinite(pv[k]) || !(pv[k] > 1e-13)) {
      throw Error{TS_ESINGULAR,
                  "coarse matrix A_" + std::to_string(c) + " is not positive definite (pivot " + std::to_string(k) +
                      " = " + std::to_string(pv[k]) + "): some affine function vanishes at every data point"};
    }
  }
}

// B_c = the explicit inverse of A_c (of its Jacobi-scaled form, scaled
// back); then level by level B_g from B_{g-1} by the steps of Alg. 7 on
// dense matrices (bottom.hip), up to the chosen level; B_g kept in FP64 and
// FP32. (The coarse solve's refinement step is left out here: formed as the
// matrix B + B (I - A_c B) it loses accuracy in the energy norm where
// kappa(A_c) is large, instead of gaining it as it does on each vector.)
static void build_bottom(Problem* P) {
  P->bottom_g = 0;
  if (g_arena) return;   // the no-allocation solve runs every level
  std::vector<int64_t> K(size_t(P->G) + 1, 0);
  std::vector<char> ok(size_t(P->G) + 1, 0);
  for (int g = P->Gc; g <= P->G; ++g) {
    K[size_t(g)] = P->lev[g].K;
    ok[size_t(g)] = P->general || P->lev[g].S64.p != nullptr;
  }
  const int gb = choose_bottom(P->opt, P->Gc, P->G, K, ok, P->general);
  if (gb == 0) return;
  const int D = P->d, nu1 = P->opt.nu1, nu2 = P->opt.nu2;
  hipStream_t s = P->stream;
  int64_t Kc = P->K1;
  DevBuf<double> Bc, T;
  Bc.alloc(size_t(Kc * Kc));
  hip_check(hipMemcpyAsync(Bc.p, P->A1inv.p, sizeof(double) * size_t(Kc * Kc), hipMemcpyDeviceToDevice, s),
            "bottom");
  for (int g = P->Gc + 1; g <= gb; ++g) {
    Level& L = P->lev[g];
    const int64_t Kf = L.K;
    const int M = int(Kf), Nc = int(Kc);
    const double* w = L.wdinv64.p;
    DevBuf<double> A, M1, X, tmp, R, Pm, Y, Z;
    A.alloc(size_t(Kf * Kf));
    R.alloc(size_t(Kc * Kf));
    Pm.alloc(size_t(Kf * Kc));
    if (P->general) {
      dense_level_general(P, g, A.p);
      restriction_dense_general(P, g, R.p);
      hip_check(launch_transpose(R.p, Kc, Kf, Pm.p, s), "bottom");
    } else {
      hip_check(launch_fill<double>(A.p, 0.0, Kf * Kf, s), "fill");
      hip_check(launch_dense_from_stencil(D, L.S64.p, L.J, Kf, A.p, s), "bottom");
      hip_check(launch_subdivision_dense(R.p, D, P->lev[g - 1].J, L.J, false, s), "bottom");
      hip_check(launch_subdivision_dense(Pm.p, D, P->lev[g - 1].J, L.J, true, s), "bottom");
    }
    tmp.alloc(size_t(Kf * Kf));
    T.alloc(size_t(Kf * Kf));
    Y.alloc(size_t(Kc * Kf));
    if (nu1 >= 1) {
      // M1 = W, then M1 += W (I - A M1) for each further sweep
      M1.alloc(size_t(Kf * Kf));
      hip_check(launch_diag_dense(w, Kf, M1.p, s), "bottom");
      for (int j = 1; j < nu1; ++j) {
        hip_check(launch_gemm64(A.p, M1.p, M, M, M, M1.p, w, 1.0, -1.0, tmp.p, s), "bottom");
        std::swap(M1, tmp);
      }
      // T = I - A M1, the residual after the pre-smoothing; Y = I' T
      if (nu1 == 1) hip_check(launch_eye_minus_scaled(A.p, w, Kf, T.p, s), "bottom");
      else hip_check(launch_gemm64(A.p, M1.p, M, M, M, nullptr, nullptr, 1.0, -1.0, T.p, s), "bottom");
      hip_check(launch_gemm64(R.p, T.p, Nc, M, M, nullptr, nullptr, 0.0, 1.0, Y.p, s), "bottom");
    } else {
      hip_check(hipMemcpyAsync(Y.p, R.p, sizeof(double) * size_t(Kc * Kf), hipMemcpyDeviceToDevice, s), "bottom");
    }
    // Z = B_{g-1} Y; X = M1 + I Z
    Z.alloc(size_t(Kc * Kf));
    hip_check(launch_gemm64(Bc.p, Y.p, Nc, M, Nc, nullptr, nullptr, 0.0, 1.0, Z.p, s), "bottom");
    X.alloc(size_t(Kf * Kf));
    hip_check(launch_gemm64(Pm.p, Z.p, M, M, Nc, nu1 >= 1 ? M1.p : nullptr, nullptr, 0.0, 1.0, X.p, s), "bottom");
    // post-smoothing: X += W (I - A X), nu2 times
    for (int j = 0; j < nu2; ++j) {
      hip_check(launch_gemm64(A.p, X.p, M, M, M, X.p, w, 1.0, -1.0, tmp.p, s), "bottom");
      std::swap(X, tmp);
    }
    if (nu1 == nu2) hip_check(launch_symmetrize(X.p, M, s), "bottom");
    hip_check(hipStreamSynchronize(s), "sync");   // the temporaries of this level are released
    Bc = std::move(X);
    Kc = Kf;
  }
  P->bottom64 = std::move(Bc);
  P->bottom32.alloc(size_t(Kc * Kc));
  hip_check(launch_round_f32(P->bottom64.p, Kc * Kc, P->bottom32.p, s), "bottom");
  hip_check(hipStreamSynchronize(s), "sync");
  P->bottom_g = gb;
  P->bottom_nu1 = nu1;
  P->bottom_nu2 = nu2;
}

void check_solve_options(const ts_options& o) {
  if (o.nu1 < 0 || o.nu2 < 0) throw Error{TS_EINVAL, "nu1, nu2 must be >= 0"};
  if (!precision_available(o.precision)) throw Error{TS_EINVAL, "unknown or unavailable precision"};
  if (!(o.tol > 0.0)) throw Error{TS_EINVAL, "tol must be > 0"};
  if (o.max_iter < 0 || o.max_refine < 0) throw Error{TS_EINVAL, "iteration limits must be >= 0"};
  if (o.preconditioner != TS_PC_MG && o.preconditioner != TS_PC_NONE && o.preconditioner != TS_PC_JACOBI)
    throw Error{TS_EINVAL, "unknown preconditioner"};
  if (o.smoother != TS_SMOOTH_JACOBI && o.smoother != TS_SMOOTH_SSOR) throw Error{TS_EINVAL, "unknown smoother"};
  if (o.smoother == TS_SMOOTH_SSOR && !(o.ssor_omega > 0.0 && o.ssor_omega < 2.0))
    throw Error{TS_EINVAL, "ssor_omega must be in (0, 2)"};
  if (o.coarse_tol < 0.0 || o.coarse_max_iter < 0) throw Error{TS_EINVAL, "coarse CG limits must be >= 0"};
  if (o.vcycle_graph != 0 && o.vcycle_graph != 1) throw Error{TS_EINVAL, "vcycle_graph must be 0 or 1"};
}

Problem* create_problem(int d, int q, const int32_t* intervals, const double* lo, const double* hi, int64_t n,
                        const double* x, const double* y, double lam, const ts_options* opt,
                        double stencil_budget) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t mem_base = g_mem.live;
  g_mem.peak = g_mem.live;
  if (d < 1 || d > kMaxDim) throw Error{TS_EINVAL, "d must be in 1..5"};
  if (!intervals || !lo || !hi || !x || !y) throw Error{TS_EINVAL, "null argument"};
  if (n < 1) throw Error{TS_EINVAL, "n must be >= 1"};
  if (!(lam > 0.0) || !std::isfinite(lam)) throw Error{TS_EINVAL, "lambda must be finite and > 0"};
  for (int p = 0; p < d; ++p) {
    if (!(lo[p] < hi[p]) || !std::isfinite(lo[p]) || !std::isfinite(hi[p]))
      throw Error{TS_EINVAL, "box must satisfy lo < hi with finite bounds"};
    if (intervals[p] < 1) throw Error{TS_EINVAL, "intervals must be >= 1"};
  }
  const int32_t* degrees = opt ? opt->degrees : nullptr;
  int32_t qs[kMaxDim];
  for (int p = 0; p < d; ++p) qs[p] = degrees ? degrees[p] : q;
  const bool general = needs_general(d, q, intervals, degrees);
  const int N = intervals[0];
  int G = 0;
  if (general) {
    // degree q_p and intervals N_p per dimension (Sec. 2.1)
    double cells = 1.0, K = 1.0, patch = 1.0;
    for (int p = 0; p < d; ++p) {
      if (qs[p] < 1 || qs[p] > kQMax) throw Error{TS_EINVAL, "degrees must be in 1..5"};
      cells *= intervals[p];
      K *= intervals[p] + qs[p];
      patch *= qs[p] + 1;
    }
    if (cells > double(1 << 30)) throw Error{TS_EINVAL, "prod N_p must not exceed 2^30 cells"};
    if (K >= 2147483647.0) throw Error{TS_EINVAL, "prod (N_p + q_p) must be < 2^31"};
    if (patch > 1024.0) throw Error{TS_EINVAL, "prod (q_p + 1) must not exceed 1024"};
    G = general_levels(d, intervals);
  } else {
    if (N < 2 || (N & (N - 1)) != 0) throw Error{TS_EINVAL, "intervals must be a power of two >= 2"};
    while ((1 << G) < N) ++G;
    if (int64_t(G) * d > 30) throw Error{TS_EINVAL, "N^d must not exceed 2^30 cells"};
    double K = std::pow(double(N + kDeg), d);
    if (K >= 2147483647.0) throw Error{TS_EINVAL, "(N+3)^d must be < 2^31"};
  }
  if (n > 2000000000LL) throw Error{TS_EINVAL, "n must be < 2e9"};

  Problem* P = new Problem();
  try {
    P->d = d;
    P->G = G;
    P->N = N;
    P->general = general;
    P->n = n;
    P->lam = lam;
    ts_default_options(&P->opt);
    if (opt) P->opt = *opt;
    check_solve_options(P->opt);
    if (P->opt.coarse_solver != TS_COARSE_DIRECT && P->opt.coarse_solver != TS_COARSE_CG)
      throw Error{TS_EINVAL, "unknown coarse solver"};
    if (P->opt.coarsest_level < 1 || P->opt.coarsest_level > G)
      throw Error{TS_EINVAL, "coarsest_level must be in 1..G = " + std::to_string(G)};
    P->Gc = P->opt.coarsest_level;
    if (P->opt.deterministic != 0 && P->opt.deterministic != 1) throw Error{TS_EINVAL, "deterministic must be 0 or 1"};
    P->det = P->opt.deterministic == 1;
    if (P->det && general)
      throw Error{TS_EINVAL, "the deterministic mode takes cubic splines on equal power-of-two grids"};
    if (P->opt.coarse_solver == TS_COARSE_DIRECT) {
      int64_t Kc = 1;
      for (int p = 0; p < d; ++p)
        Kc *= general ? (intervals[p] >> (G - P->Gc)) + qs[p] : (int64_t(1) << P->Gc) + kDeg;
      if (Kc > kMaxDirectCoarse)
        throw Error{TS_EINVAL, "the direct coarse solver takes K_c <= " + std::to_string(kMaxDirectCoarse) +
                                   " coefficients (K_c = " + std::to_string(Kc) + "); use TS_COARSE_CG"};
    }
    if (P->opt.omega_fixed <= 0.0 && !(P->opt.omega_scale > 0.0 && P->opt.omega_scale < 2.0))
      throw Error{TS_EINVAL, "omega_scale must be in (0, 2)"};
    hip_check(hipGetDevice(&P->device), "hipGetDevice");
    if (P->opt.stream) {
      P->stream = static_cast<hipStream_t>(P->opt.stream);
    } else if (g_arena) {
      P->stream = nullptr;   // no resources are created in the no-allocation mode
    } else {
      hip_check(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking), "stream");
      P->own_stream = true;
    }
    if (g_arena) {
      // host scalars in ordinary thread-local memory; readbacks synchronise the stream
      static thread_local double host_slots[kSlots];
      P->host_slots = host_slots;
      P->pinned_slots = false;
    } else {
      hip_check(hipHostMalloc(reinterpret_cast<void**>(&P->host_slots), sizeof(double) * kSlots), "pinned");
      hip_check(hipEventCreateWithFlags(&P->slots_ready, hipEventDisableTiming), "event");
    }
    P->slots.alloc(kSlots);
    P->partial.alloc(3 * kMaxPartials);   // three rows of per-block partials
    P->flag.alloc(1);
    for (int p = 0; p < d; ++p) {
      P->box.lo[p] = lo[p];
      P->box.hi[p] = hi[p];
      P->box.inv_h[p] = double(N) / (hi[p] - lo[p]);
    }
    P->box.G = G;
    hipStream_t st = P->stream;

    // --- bin, validate, sort, place (points in Morton order of their cell;
    // the general form: in C order)
    if (general) {
      setup_general_points(P, intervals, qs, lo, hi, x, y);
    } else {
      DevBuf<uint32_t> key0, key1, idx0, idx1;
      key0.alloc(size_t(n));
      key1.alloc(size_t(n));
      idx0.alloc(size_t(n));
      idx1.alloc(size_t(n));
      hip_check(launch_fill<int>(P->flag.p, 0, 1, st), "fill");
      hip_check(launch_bin(d, x, n, P->box, key0.p, idx0.p, P->flag.p, st), "bin");
      hip_check(launch_check_finite(y, n, P->flag.p, st), "check y");
      int flag = 0;
      hip_check(hipMemcpyAsync(&flag, P->flag.p, sizeof(int), hipMemcpyDeviceToHost, st), "flag");
      hip_check(hipStreamSynchronize(st), "sync");
      if (flag & 2) throw Error{TS_EINVAL, "x contains non-finite values"};
      if (flag & 4) throw Error{TS_EINVAL, "some points lie outside [lo, hi]"};
      if (flag & 1) throw Error{TS_EINVAL, "y contains non-finite values"};
      size_t tmp_bytes = 0;
      hip_check(sort_pairs(key0.p, key1.p, idx0.p, idx1.p, n, G * d, nullptr, &tmp_bytes, st), "sort size");
      DevBuf<unsigned char> tmp;
      tmp.alloc(tmp_bytes + 16);
      hip_check(sort_pairs(key0.p, key1.p, idx0.p, idx1.p, n, G * d, tmp.p, &tmp_bytes, st), "sort");
      P->t64.alloc(size_t(n) * d);
      P->t32.alloc(size_t(n) * d);
      P->cell.alloc(size_t(n));
      P->ys.alloc(size_t(n));
      hip_check(launch_place(d, x, y, idx1.p, n, P->box, P->t64.p, P->t32.p, P->cell.p, P->ys.p, st), "place");
      const int64_t ncells = int64_t(1) << (G * d);
      P->off.alloc(size_t(ncells + 1));
      hip_check(launch_offsets(key1.p, n, ncells, P->off.p, st), "offsets");
      hip_check(hipStreamSynchronize(st), "sync");
      P->mkey = std::move(key1);
    }

    // --- data-term work split
    // (the point pass stages at most kMaxPointsPerBlock[d] points per workgroup)
    const int ppb_max = kMaxPointsPerBlock[d];
    if (P->opt.points_per_block > 0) {
      P->ppb = std::max(64, std::min(ppb_max, P->opt.points_per_block));
    } else {
      // the largest power of two <= n / 16384, within [256, ppb_max]
      // (measured best on MI355X: 256 at 2e6 points, 512 at 1e7 and 2e7)
      int64_t ppb = 256;
      while (ppb * 2 <= n / 16384) ppb *= 2;
      P->ppb = int(std::max<int64_t>(std::min(256, ppb_max), std::min<int64_t>(ppb_max, ppb)));
    }

    // --- levels g = 1..G (N_g = 2^g)
    P->lev.resize(G + 1);
    const int64_t KG = [&] {
      int64_t K = 1;
      for (int p = 0; p < d; ++p) K *= general ? intervals[p] + qs[p] : N + kDeg;
      return K;
    }();
    for (int g = 1; g <= G; ++g) {
      Level& L = P->lev[g];
      L.g = g;
      if (general) {
        // sizes on every level (ts_num_coeffs), the banded factors from level c on
        if (g < P->Gc) {
          L.K = 1;
          for (int p = 0; p < d; ++p) L.K *= (intervals[p] >> (G - g)) + qs[p];
          continue;
        }
        setup_general_level(P, g, lo, hi);
      } else {
        L.N = 1 << g;
        L.J = L.N + kDeg;
        L.K = 1;
        for (int p = 0; p < d; ++p) L.K *= L.J;
        L.tb = std::min(kTileBits[d], g);
        if (g < P->Gc) continue;   // below the coarsest level: sizes only
        std::vector<double> band(size_t(d) * 3 * L.J * 7);
        for (int p = 0; p < d; ++p) {
          std::vector<double> b1;
          gram_band(lo[p], hi[p], L.N, b1);
          std::copy(b1.begin(), b1.end(), band.begin() + size_t(p) * 3 * L.J * 7);
        }
        std::vector<float> bandf(band.begin(), band.end());
        L.band64.alloc(band.size());
        L.band32.alloc(band.size());
        hip_check(hipMemcpyAsync(L.band64.p, band.data(), band.size() * 8, hipMemcpyHostToDevice, st), "upload");
        hip_check(hipMemcpyAsync(L.band32.p, bandf.data(), bandf.size() * 4, hipMemcpyHostToDevice, st), "upload");
      }
      L.diag.alloc(size_t(L.K));
      L.wdinv64.alloc(size_t(L.K));
      L.wdinv32.alloc(size_t(L.K));
      L.a64.alloc(size_t(L.K));
      L.b64.alloc(size_t(L.K));
      L.t64.alloc(size_t(L.K));
      L.a32.alloc(size_t(L.K));
      L.b32.alloc(size_t(L.K));
      L.t32.alloc(size_t(L.K));
      hip_check(hipStreamSynchronize(st), "sync");   // host band vectors go out of scope
    }
    P->lamS64.alloc(size_t(6 * KG));
    P->lamS32.alloc(size_t(6 * KG));
    P->xfer64.alloc(size_t(2 * KG));
    P->xfer32.alloc(size_t(2 * KG));
    P->vb.alloc(size_t(KG));
    P->vr.alloc(size_t(KG));
    P->vz.alloc(size_t(KG));
    P->vp.alloc(size_t(KG));
    P->vv.alloc(size_t(KG));
    P->r32.alloc(size_t(KG));
    P->z32.alloc(size_t(KG));
    P->p32.alloc(size_t(KG));
    P->v32.alloc(size_t(KG));
    P->d32.alloc(size_t(KG));

    // --- assembled stencils for the levels where they pay (same A_g), and
    // the point pass's work lists on the other levels, built on a host
    // thread meanwhile (the general form runs matrix-free on every level)
    if (!general) {
      const double budget = stencil_budget_for(stencil_budget);
      std::vector<char> want(size_t(G) + 1, 0);
      bool matrix_free = false;
      const int Gc = P->Gc;
      // work lists on the levels applied matrix-free; in the deterministic
      // mode on every level (the setup's diagonal and right-hand-side passes
      // take them too)
      std::vector<char> listed(size_t(G) + 1, 0);
      for (int g = Gc; g <= G; ++g) {
        want[size_t(g)] = want_stencil(d, P->lev[g].J, n, P->opt.stencil_mode, budget);
        listed[size_t(g)] = !want[size_t(g)] || P->det;
        matrix_free = matrix_free || listed[size_t(g)];
      }
      std::vector<int32_t> off_h;
      if (matrix_free) {
        off_h.resize(size_t((int64_t(1) << (G * d)) + 1));
        hip_check(hipMemcpyAsync(off_h.data(), P->off.p, off_h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "download");
        hip_check(hipStreamSynchronize(st), "sync");
      }
      std::vector<int> tbs(size_t(G) + 1);
      for (int g = 1; g <= G; ++g) tbs[size_t(g)] = P->lev[g].tb;
      const int64_t ppb = P->ppb;
      auto lists = std::async(std::launch::async, [&listed, &off_h, tbs, ppb, d, G, Gc]() {
        std::vector<WorkListHost> r(size_t(G) + 1);
        for (int g = Gc; g <= G; ++g)
          if (listed[size_t(g)]) r[size_t(g)] = make_worklist(d, G, g, tbs[size_t(g)], ppb, off_h);
        return r;
      });
      // finest first: each level's moments give the next coarser level's
      DevBuf<double> mom;
      for (int g = G; g >= Gc; --g) {
        if (!want[size_t(g)]) { mom.reset(); continue; }
        build_stencil(P, g, mom, g > Gc && want[size_t(g) - 1]);
      }
      const std::vector<WorkListHost> wl = lists.get();
      for (int g = Gc; g <= G; ++g)
        if (listed[size_t(g)]) upload_worklist(P, g, wl[size_t(g)]);
      if (P->det) {
        // the stored patches of the largest level (applies run one at a time)
        size_t part = 1;
        for (int g = Gc; g <= G; ++g) {
          size_t patch = 1;
          for (int p = 0; p < d; ++p) patch *= size_t((1 << P->lev[g].tb) + kDeg);
          part = std::max(part, (wl[size_t(g)].chunks.size() - 1) * patch);
        }
        P->det_part.alloc(part);
      }
    }

    // --- Jacobi diagonals and damping (Alg. 5, Alg. 6)
    for (int g = P->Gc; g <= G; ++g) compute_diag(P, g);
    for (int g = P->Gc + 1; g <= G; ++g) {
      Level& L = P->lev[g];
      if (P->opt.omega_fixed > 0.0) {
        L.omega = P->opt.omega_fixed;
      } else {
        L.theta = lanczos_theta(P, g, std::max(1, P->opt.lanczos_steps));
        L.omega = P->opt.omega_scale / L.theta;
      }
      hip_check(launch_wdinv(L.diag.p, L.omega, L.wdinv64.p, L.wdinv32.p, L.K, st), "wdinv");
    }

    {   // D_G^-1 for the Jacobi preconditioner
      DevBuf<float> unused;
      unused.alloc(size_t(KG));
      P->dinv_fine.alloc(size_t(KG));
      hip_check(launch_wdinv(P->lev[G].diag.p, 1.0, P->dinv_fine.p, unused.p, KG, st), "dinv");
      hip_check(hipStreamSynchronize(st), "sync");
    }

    // --- coarse level (Sec. 3.2.4)
    build_coarse(P);
    build_bottom(P);
    hip_check(hipStreamSynchronize(st), "sync");
    P->applies = 0;
    P->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    P->mem_resident = g_mem.live - mem_base;
    P->mem_peak = g_mem.peak - mem_base;
    return P;
  } catch (...) {
    delete P;
    throw;
  }
}

Problem::~Problem() {
  (void)hipStreamSynchronize(stream);   // also the null stream of the no-allocation mode
  for (Captured& c : vgraph)
    if (c.exec) (void)hipGraphExecDestroy(c.exec);
  lev.clear();
  if (host_slots && pinned_slots) (void)hipHostFree(host_slots);
  if (slots_ready) (void)hipEventDestroy(slots_ready);
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

}  // namespace tsmg
