// Internal state of one smoothing problem (host-side view of device memory).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/tsmg.h"
#include "general.h"
#include "launch.h"

namespace tsmg {

struct Error {
  ts_status code;
  std::string msg;
};

void hip_check(hipError_t e, const char* what);

// Precision modes this build solves in (TS_MIXED_BF16 is reserved).
inline bool precision_available(int p) {
  return p == TS_FP64 || p == TS_MIXED_FP32 || p == TS_MIXED_FP32_VCYCLE;
}
// Checks of the solve-time option fields shared by ts_create and
// ts_set_options; throws Error{TS_EINVAL}.
void check_solve_options(const ts_options& o);
// Largest coarsest-level size the direct coarse solver inverts.
constexpr int64_t kMaxDirectCoarse = 4096;
void set_error(const std::string& m);

// Device bytes held by DevBuf objects allocated on this thread (live) and
// the high-water mark since the last reset; a problem records both around
// its setup.
struct MemCount {
  int64_t live = 0;
  int64_t peak = 0;
};
extern thread_local MemCount g_mem;

// Device memory cache of the library (per device, shared by all problems
// and threads). pool_alloc returns a block of at least `bytes`, reusing one
// released earlier when one of a close size is cached, else from hipMalloc
// (after emptying the cache if hipMalloc fails); throws Error{TS_ENOMEM}.
// pool_release caches the block, or frees it when the cache is full. A
// block may be released only once no queued device work uses it.
void* pool_alloc(size_t bytes);
void pool_release(void* p);

// Bump allocator over a caller-provided device region. While a thread has
// g_arena set, pool_alloc on that thread carves blocks from it (256-byte
// aligned) and throws Error{TS_EINVAL} once it is exhausted; pool_release
// ignores blocks inside any region registered with register_arena_region.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
};
extern thread_local Arena* g_arena;
void register_arena_region(void* base, size_t bytes);

// Owning device buffer, returned to the cache on destruction. Every owner
// synchronises the stream its buffers were used on before releasing them;
// a buffer released while an exception unwinds is freed with hipFree
// instead, which waits for the device.
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { reset(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { reset(); }
  void alloc(size_t count) {
    reset();
    if (count == 0) count = 1;
    p = static_cast<T*>(pool_alloc(count * sizeof(T)));
    n = count;
    g_mem.live += int64_t(count * sizeof(T));
    if (g_mem.live > g_mem.peak) g_mem.peak = g_mem.live;
  }
  void reset() {
    if (p) {
      pool_release(p);
      g_mem.live -= int64_t(n * sizeof(T));
    }
    p = nullptr;
    n = 0;
  }
};

struct Level {
  int g = 0, N = 0, J = 0;
  int64_t K = 0;
  int tb = 0;                      // tile side 2^tb cells per dimension in the point pass
  double theta = 0.0, omega = 0.0; // Lanczos estimate and Jacobi damping
  DevBuf<double> band64;           // [d][3][J][7] banded M, G1, G2 per dimension
  DevBuf<float> band32;
  DevBuf<double> diag;             // diag(A_g)
  DevBuf<double> wdinv64;          // omega_g / diag(A_g)
  DevBuf<float> wdinv32;
  DevBuf<double> a64, b64, t64;    // V-cycle iterate, right-hand side, A x work vector
  DevBuf<float> a32, b32, t32;
  bool stencil = false;            // A_g assembled as a 7^d-point stencil
  DevBuf<double> S64;              // [(7^d+1)/2][K] offset-major stencil, upper half of the offsets
  DevBuf<float> S32;
  // work list of the point pass (levels applied matrix-free)
  GenLevel gl{};                   // general form: sizes, degrees, strides, band offsets
  DevBuf<int32_t> wl_first;        // [workgroups + 1]
  DevBuf<int4> wl_chunks;          // [chunks + 1]
  DevBuf<uint32_t> wl_items;       // [items]
  int wl_groups = 0;
  DevBuf<int32_t> det_tile_first;  // deterministic mode: [tiles + 1] first chunk of each tile
};

constexpr int kSlots = 80;
constexpr int kLanczosSlot0 = 16;   // slots 16.. hold the Lanczos scalars during setup

struct Problem {
  int device = 0;
  int d = 0, G = 0, N = 0;
  int64_t n = 0;
  double lam = 0.0;
  ts_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  BoxArgs box{};
  int ppb = 256;

  // general form (degree and intervals per dimension, general_setup.cpp): the
  // points are sorted by their finest cell in C order instead, and every
  // level is applied matrix-free by the general kernels
  bool general = false;
  GenBox gbox{};
  int gq[kMaxDim] = {};
  DevBuf<int32_t> gcell;    // [d][n] finest cell per dimension

  // points in Morton order of their finest cell
  DevBuf<double> t64;       // [d][n] position inside the finest cell
  DevBuf<float> t32;        // [d][n]
  DevBuf<uint32_t> cell;    // [n] finest cell, C order
  DevBuf<uint32_t> mkey;    // [n] finest cell, Morton order (sorted)
  DevBuf<double> ys;        // [n] responses
  DevBuf<int32_t> off;      // [N^d + 1] Morton cell offsets

  std::vector<Level> lev;   // index 1..G
  DevBuf<double> lamS64;    // 6 K_G: two sets of (T0, T1, T2)
  DevBuf<float> lamS32;
  DevBuf<double> xfer64;    // 2 K_G: transfer intermediates
  DevBuf<float> xfer32;
  int Gc = 1;               // coarsest level c of the V-cycle (Sec. 3.2.4)
  DevBuf<double> A1;        // K_c x K_c coarse matrix (for the refinement step)
  DevBuf<double> A1inv;     // K_c x K_c inverse of the coarse matrix
  DevBuf<double> cwork;     // 2 K_c coarse-solve work space
  int K1 = 0;               // K_c
  // coarse CG (TS_COARSE_CG): D_c^-1 and the CG vectors of level c
  DevBuf<double> cdinv, cx, cr, cz, cp, cv;
  int64_t coarse_iters = 0; // coarse CG iterations of the last solve
  // the V-cycle from level bottom_g down as one dense operator (0: none),
  // assembled for the smoothing counts bottom_nu1, bottom_nu2
  int bottom_g = 0, bottom_nu1 = 0, bottom_nu2 = 0;
  DevBuf<double> bottom64;  // K x K, K = K_{bottom_g}
  DevBuf<float> bottom32;

  // solver vectors on the finest level
  DevBuf<double> vb, vr, vz, vp, vv;
  DevBuf<double> dinv_fine;      // D_G^-1 (TS_PC_JACOBI)
  DevBuf<float> r32, z32, p32, v32, d32;

  DevBuf<double> slots;     // device scalars
  DevBuf<double> partial;   // reduction partials [3][kMaxPartials]
  bool det = false;         // opt.deterministic: reproducible point passes and moments
  DevBuf<double> det_part;  // deterministic point pass: [chunks][patch] of the largest level
  DevBuf<int> flag;
  double* host_slots = nullptr;
  bool pinned_slots = true;   // host_slots from hipHostMalloc (else caller-owned host memory)

  // V-cycles of a solve replayed from captured HIP graphs, one per kind of
  // call (precision, first sweep already written); key: the pointers and
  // options the capture baked in; applies: operator applies per replay
  struct Captured {
    hipGraphExec_t exec = nullptr;
    uint64_t key = 0;
    int64_t applies = 0;
  };
  Captured vgraph[4];

  double setup_s = 0.0;
  int64_t applies = 0;
  std::vector<double> history;   // residual history of the last solve
  int64_t mem_resident = 0;   // device bytes held after setup
  int64_t mem_peak = 0;       // most device bytes held during setup

  double* slot(int i);
  void read_slots(int first, int count, double* host);
  // read_slots in two halves: queue the copy (and an event) on the stream,
  // then wait for that event and read; work queued in between overlaps the
  // host's wait
  void copy_slots(int first, int count);
  void wait_slots(int first, int count, double* host);
  hipEvent_t slots_ready = nullptr;
  ~Problem();
};

// stencil_budget > 0 caps the bytes of assembled stencils per level at that
// value; 0 takes min(16 GB, 40% of the free device memory).
Problem* create_problem(int d, int q, const int32_t* intervals, const double* lo, const double* hi, int64_t n,
                        const double* x, const double* y, double lam, const ts_options* opt,
                        double stencil_budget = 0.0);

// Upper estimate of the device bytes create_problem and a solve hold at
// their peak, for the same arguments (the points themselves excluded).
int64_t footprint_bytes(int d, int N, int64_t n, const ts_options& opt, double stencil_budget);

template <typename T> void apply_op(Problem* P, int g, const T* c, T* out);
template <typename T> void prolong_op(Problem* P, int g, const T* e, T* out, bool subtract);
template <typename T>
void restrict_op(Problem* P, int g, const T* r, T* out, const T* sub, const T* w0 = nullptr, T* a0 = nullptr);
template <typename T> void coarse_op(Problem* P, const T* b, T* x);
// Arguments of the point pass on level g (its work list and, in the
// deterministic mode, the stored-patch area) for input c and output out.
DataArgs data_args(Problem* P, int g, bool fp32, const void* c, void* out);
// One V-cycle on level g from a zero start; pre_done: the first Jacobi sweep
// (alpha = w .* b) was already written by the restriction that produced b.
template <typename T> void vcycle_op(Problem* P, int g, const T* b, T* alpha, bool pre_done = false);
// Where the first Jacobi sweep of a V-cycle on level g with output alpha
// lands when it is the plain product w .* b (which the kernel producing b may
// then write instead, passing pre_done); null when it is not.
template <typename T> T* first_sweep_target(Problem* P, int g, T* alpha);
// The level whose V-cycle the dense operator replaces under the current
// options, or 0.
int bottom_level(const Problem* P);
template <typename T> void profile_apply(Problem* P, int g, int reps, double* ms_lambda, double* ms_data);
template <typename TX, typename TY> void dot_op(Problem* P, const TX* x, const TY* y, int64_t K, int slot);

ts_status solve(Problem* P, double* alpha, int use_start, ts_solve_info* info);

// The general form (general_setup.cpp).
bool needs_general(int d, int q, const int32_t* N, const int32_t* degrees);
int general_levels(int d, const int32_t* N);
// Upper estimate of the peak device bytes of a general-form problem.
int64_t footprint_general(int d, int q, const int32_t* N, int64_t n, const ts_options& opt);
void setup_general_points(Problem* P, const int32_t* N, const int32_t* q, const double* lo, const double* hi,
                          const double* x, const double* y);
void setup_general_level(Problem* P, int g, const double* lo, const double* hi);
template <typename T> void apply_general(Problem* P, int g, const T* c, T* out);
template <typename T>
void transfer_general(Problem* P, int g, bool prolong, const T* in, T* out, const T* sub, bool subtract);
template <typename T>
void profile_general(Problem* P, int g, T* c, T* out, int reps, hipEvent_t e0, hipEvent_t e1, hipEvent_t e2);
void rhs_general(Problem* P, double* b);
void diag_general(Problem* P, int g);
void coarse_matrix_general(Problem* P, double* A);
// A_g of a general level, dense (lam Lambda_g + Phi_g'Phi_g from the points).
void dense_level_general(Problem* P, int g, double* A);
// The dense restriction I_g' (K_{g-1} x K_g) of a general level.
void restriction_dense_general(Problem* P, int g, double* R);
// The level from which the V-cycle is assembled as one dense operator (0:
// none), given the level sizes K[g] and which levels can be assembled.
int choose_bottom(const ts_options& o, int Gc, int G, const std::vector<int64_t>& K, const std::vector<char>& ok,
                  bool general);
void eval_general(Problem* P, const double* alpha, int64_t m, const double* xq, double* yq);

}  // namespace tsmg

struct ts_problem {
  tsmg::Problem* impl;
};
