// Krylov drivers: MGCG (Alg. 8) in FP64 and the mixed-precision refinement
// loop around an FP32 MGCG. Scalars stay on the device; each iteration reads
// back p'v and r'r once for the breakdown and stopping tests.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <utility>

#include "problem.h"

namespace tsmg {

namespace {

enum Slot : int { kScratch = 0, kBB = 1, kRZa = 2, kRZb = 3, kPV = 4, kRR = 5, kRR64 = 6, kRZo = 7 };

void rhs_into(Problem* P, double* b) {
  if (P->general) {
    rhs_general(P, b);
    return;
  }
  const int64_t K = P->lev[P->G].K;
  hip_check(launch_fill<double>(b, 0.0, K, P->stream), "fill");
  hip_check(launch_data(P->d, false, kRhs, data_args(P, P->G, false, nullptr, b), P->stream), "rhs");
}

// r = b - A alpha (FP64); uses v as work space.
void true_residual(Problem* P, const double* alpha, const double* b, double* r, double* v) {
  const int64_t K = P->lev[P->G].K;
  apply_op<double>(P, P->G, alpha, v);
  hip_check(launch_residual<double>(r, v, b, K, P->stream), "residual");       // r = Av - b
  hip_check(launch_scale_copy<double, double>(r, r, K, -1.0, nullptr, P->stream), "negate");
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// TSMG_PROGRESS=k in the environment: every k-th iteration of a solve prints
// its iteration count and recursive relative residual to stderr (for long
// solves run under a watchdog that expects output).
int progress_every() {
  const char* e = std::getenv("TSMG_PROGRESS");
  const int k = e ? std::atoi(e) : 0;
  return k > 0 ? k : 0;
}

void report(int every, const char* mode, int it, double rel) {
  if (every > 0 && it % every == 0) {
    std::fprintf(stderr, "tsmg %s iteration %d rel. residual %.3e\n", mode, it, rel);
    std::fflush(stderr);
  }
}

// The V-cycle of a solve as a captured HIP graph (vcycle_graph set): its
// kernels are recorded once (per kind of call and per set of pointers and
// options they bake in) and then replayed each iteration with one launch.
// Only kernel launches are recorded: no memsets, no host reads. Not used on
// the null stream, with the no-allocation arena (instantiation may
// allocate) or with the CG coarse solver (it reads its residual on the host).
bool capture_usable(const Problem* P) {
  return P->opt.vcycle_graph == 1 && P->stream != nullptr && g_arena == nullptr &&
         P->opt.coarse_solver != TS_COARSE_CG;
}

uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}

uint64_t capture_key(const Problem* P, const void* in, const void* out, const void* aux) {
  uint64_t h = 0;
  double om = P->opt.ssor_omega;
  uint64_t omb = 0;
  static_assert(sizeof(om) == sizeof(omb), "double is 64 bits");
  std::memcpy(&omb, &om, sizeof(omb));
  for (uint64_t v : {uint64_t(reinterpret_cast<uintptr_t>(in)), uint64_t(reinterpret_cast<uintptr_t>(out)),
                     uint64_t(reinterpret_cast<uintptr_t>(aux)), uint64_t(P->opt.nu1), uint64_t(P->opt.nu2),
                     uint64_t(P->opt.smoother), omb, uint64_t(bottom_level(P)),
                     uint64_t(reinterpret_cast<uintptr_t>(P->stream))})
    h = mix(h, v);
  return h | 1;   // never 0, the key of an empty entry
}

template <typename F>
void run_captured(Problem* P, int which, uint64_t key, F&& body) {
  if (!capture_usable(P)) {
    body();
    return;
  }
  Problem::Captured& c = P->vgraph[which];
  if (!c.exec || c.key != key) {
    if (c.exec) {
      hip_check(hipStreamSynchronize(P->stream), "sync");   // no replay of the old graph is in flight
      hip_check(hipGraphExecDestroy(c.exec), "graph destroy");
      c.exec = nullptr;
    }
    const int64_t a0 = P->applies;
    hip_check(hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
      body();
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(P->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hipGraph_t g = nullptr;
    hip_check(hipStreamEndCapture(P->stream, &g), "end capture");
    const hipError_t e = hipGraphInstantiate(&c.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    hip_check(e, "graph instantiate");
    c.key = key;
    c.applies = P->applies - a0;
    P->applies = a0;
  }
  hip_check(hipGraphLaunch(c.exec, P->stream), "graph launch");
  P->applies += c.applies;
}

}  // namespace

void rhs_op(Problem* P, double* b) { rhs_into(P, b); }

// z = B r: one V-cycle in FP64, or (pc32) in FP32 on r / ||r|| with the
// result scaled back (slot rr holds ||r||^2); with TS_PC_NONE z = r (plain
// CG), with TS_PC_JACOBI z = D^-1 r.
static void precondition(Problem* P, bool pc32, const double* r, double* z, int rr, bool pre_done = false) {
  const int G = P->G;
  const int64_t K = P->lev[G].K;
  if (P->opt.preconditioner == TS_PC_NONE) {
    hip_check(launch_scale_copy<double, double>(r, z, K, 1.0, nullptr, P->stream), "copy");
    return;
  }
  if (P->opt.preconditioner == TS_PC_JACOBI) {
    hip_check(launch_mul(P->dinv_fine.p, r, z, K, P->stream), "jacobi precondition");
    return;
  }
  if (!pc32) {
    run_captured(P, pre_done ? 1 : 0, capture_key(P, r, z, nullptr),
                 [&] { vcycle_op<double>(P, G, r, z, pre_done); });
    return;
  }
  run_captured(P, 2, capture_key(P, r, z, P->slot(rr)), [&] {
    hip_check(launch_scale_copy<double, float>(r, P->r32.p, K, 1.0, P->slot(rr), P->stream), "to fp32");
    vcycle_op<float>(P, G, P->r32.p, P->z32.p);
    hip_check(launch_scale_mul(P->z32.p, z, K, P->slot(rr), P->stream), "to fp64");
  });
}

// Alg. 8 in FP64. With pc32 the V-cycle runs in FP32; then, and when the
// coarse level is solved by an inner CG (a preconditioner that is not
// exactly linear), the direction update takes the flexible form
// beta = r'(z - z_old) / r_old'z_old, which tolerates the inexactness; the
// Krylov recurrences and every operator apply stay FP64.
static ts_status solve_fp64(Problem* P, double* alpha, int use_start, ts_solve_info* info, bool pc32 = false) {
  const bool flex = pc32 || (P->opt.preconditioner == TS_PC_MG && P->opt.coarse_solver == TS_COARSE_CG);
  const int G = P->G;
  const int64_t K = P->lev[G].K;
  hipStream_t st = P->stream;
  double *b = P->vb.p, *r = P->vr.p, *z = P->vz.p, *p = P->vp.p, *v = P->vv.p;
  rhs_into(P, b);
  dot_op<double, double>(P, b, b, K, kBB);
  double bb;
  P->read_slots(kBB, 1, &bb);
  if (!std::isfinite(bb)) throw Error{TS_EBREAKDOWN, "right-hand side is not finite"};
  if (bb == 0.0) {
    hip_check(launch_fill<double>(alpha, 0.0, K, st), "fill");
    info->converged = 1;
    info->rel_residual = 0.0;
    P->history.assign(1, 0.0);
    return TS_OK;
  }
  const double bnorm = std::sqrt(bb);
  double rel_true = 1.0;
  if (use_start) {
    true_residual(P, alpha, b, r, v);
    dot_op<double, double>(P, r, r, K, kRR);
    double rr0;
    P->read_slots(kRR, 1, &rr0);
    rel_true = std::sqrt(rr0) / bnorm;
  } else {
    hip_check(launch_fill<double>(alpha, 0.0, K, st), "fill");
    hip_check(launch_scale_copy<double, double>(b, r, K, 1.0, nullptr, st), "copy");
  }
  P->history.assign(1, rel_true);
  const double tol = P->opt.tol;
  const int every = progress_every();
  int total = 0, restarts = 0;
  if (rel_true <= tol) {
    info->iterations = 0;
    info->refinements = 0;
    info->rel_residual = rel_true;
    info->converged = 1;
    return TS_OK;
  }
  // where the step kernel can write the first sweep of the next V-cycle
  double* zf = (!pc32 && P->opt.preconditioner == TS_PC_MG) ? first_sweep_target<double>(P, G, z) : nullptr;
  for (;;) {
    int sa = kRZa, sb = kRZb;
    if (pc32) dot_op<double, double>(P, r, r, K, kRR);
    precondition(P, pc32, r, z, kRR);
    hip_check(launch_scale_copy<double, double>(z, p, K, 1.0, nullptr, st), "copy");
    dot_op<double, double>(P, r, z, K, sa);
    // the first stage of p'v and of r'z (row 2 of the partials); their
    // second stages run inside the kernels that use them
    double* dpart = P->partial.p + 2 * kMaxPartials;
    int nb = 0;
    while (total < P->opt.max_iter) {
      apply_op<double>(P, G, p, v);
      hip_check(launch_dot_partial<double, double>(p, v, K, dpart, &nb, st), "dot");
      // the step (p'v summed in it) with r'r, for the flexible update
      // r_new' z_old, and the first Jacobi sweep of the V-cycle that follows
      hip_check(launch_cg_step_norms(alpha, r, p, v, flex ? z : nullptr, K, P->slot(sa), P->slot(kPV), P->partial.p,
                                     P->slot(kRR), P->slot(kRZo), zf ? P->lev[G].wdinv64.p : nullptr, zf, dpart, nb,
                                     st),
                "cg step");
      P->copy_slots(kPV, 2);
      // the next V-cycle is queued before the host reads the residual, so the
      // device does not idle during the readback; after the last iteration
      // it is wasted (z is not used again)
      precondition(P, pc32, r, z, kRR, zf != nullptr);
      double h[2];
      P->wait_slots(kPV, 2, h);
      ++total;
      if (!finite_pos(h[0]) || !std::isfinite(h[1]))
        throw Error{TS_EBREAKDOWN, "CG breakdown: p'Ap = " + std::to_string(h[0])};
      report(every, pc32 ? "vcycle32" : "fp64", total, std::sqrt(h[1]) / bnorm);
      P->history.push_back(std::sqrt(h[1]) / bnorm);
      if (std::sqrt(h[1]) / bnorm <= tol) break;
      // r'z summed in the direction update (flexible: minus r_new' z_old)
      hip_check(launch_dot_partial<double, double>(r, z, K, dpart, &nb, st), "dot");
      hip_check(launch_p_update_sum(p, z, K, P->slot(sb), dpart, nb, flex ? P->slot(kRZo) : nullptr, P->slot(sa), st),
                "p update");
      std::swap(sa, sb);
    }
    // confirm with the true FP64 residual; restart from it if the recursive
    // residual drifted below the tolerance first
    true_residual(P, alpha, b, r, v);
    dot_op<double, double>(P, r, r, K, kRR);
    double rr;
    P->read_slots(kRR, 1, &rr);
    rel_true = std::sqrt(rr) / bnorm;
    if (rel_true <= tol || total >= P->opt.max_iter || restarts >= 5) break;
    P->history.push_back(rel_true);   // the restart begins from the true residual
    ++restarts;
  }
  info->iterations = total;
  info->refinements = restarts;
  info->rel_residual = rel_true;
  info->converged = rel_true <= tol;
  return info->converged ? TS_OK : TS_ENOTCONV;
}

// Mixed precision: the CG recurrences, the operator applies and the V-cycle
// run in FP32 on the residual scaled by 1/||b||, with FP64 dot products. The
// FP32 correction is accumulated separately; whenever the FP32 residual has
// dropped by the factor inner_tol since the last update (or CG would stop),
// the correction is added to alpha in FP64, the true residual b - A alpha is
// recomputed with the FP64 operator and replaces the FP32 one, and the search
// direction is kept (CG with reliable updates: iterative refinement that does
// not restart the Krylov space). A non-positive p'Ap in FP32 (kappa(A) beyond
// single precision) forces an update that takes the V-cycle correction and
// restarts the direction.
static ts_status solve_mixed(Problem* P, double* alpha, int use_start, ts_solve_info* info) {
  const int G = P->G;
  const int64_t K = P->lev[G].K;
  hipStream_t st = P->stream;
  double *b = P->vb.p, *r = P->vr.p, *v = P->vv.p;
  float *rin = P->r32.p, *z = P->z32.p, *p = P->p32.p, *w = P->v32.p, *dl = P->d32.p;
  rhs_into(P, b);
  dot_op<double, double>(P, b, b, K, kBB);
  double bb;
  P->read_slots(kBB, 1, &bb);
  if (!std::isfinite(bb)) throw Error{TS_EBREAKDOWN, "right-hand side is not finite"};
  if (bb == 0.0) {
    hip_check(launch_fill<double>(alpha, 0.0, K, st), "fill");
    info->converged = 1;
    info->rel_residual = 0.0;
    return TS_OK;
  }
  const double bnorm = std::sqrt(bb);
  const double tol = P->opt.tol;
  const double delta = (P->opt.inner_tol > 0.0 && P->opt.inner_tol < 1.0) ? P->opt.inner_tol : 0.1;
  const int every = progress_every();
  if (use_start) {
    true_residual(P, alpha, b, r, v);
  } else {
    hip_check(launch_fill<double>(alpha, 0.0, K, st), "fill");
    hip_check(launch_scale_copy<double, double>(b, r, K, 1.0, nullptr, st), "copy");
  }
  dot_op<double, double>(P, r, r, K, kRR64);
  double rr;
  P->read_slots(kRR64, 1, &rr);
  double rel = std::sqrt(rr) / bnorm;
  P->history.assign(1, rel);
  int total = 0, updates = 0;
  if (!(rel <= tol)) {
    if (!std::isfinite(rel)) throw Error{TS_EBREAKDOWN, "residual is not finite"};
    hip_check(launch_scale_copy<double, float>(r, rin, K, 1.0 / bnorm, nullptr, st), "to fp32");
    hip_check(launch_fill<float>(dl, 0.0f, K, st), "fill");
    double rmax = rel;        // FP32 residual norm (relative to ||b||) at the last update
    bool fresh = true;        // dl is zero and p = z (first step since a (re)start)
    int sa = kRZa, sb = kRZb;
    run_captured(P, 3, capture_key(P, rin, z, nullptr), [&] { vcycle_op<float>(P, G, rin, z); });
    hip_check(launch_scale_copy<float, float>(z, p, K, 1.0, nullptr, st), "copy");
    dot_op<float, float>(P, rin, z, K, sa);
    for (;;) {
      apply_op<float>(P, G, p, w);
      dot_op<float, float>(P, p, w, K, kPV);
      hip_check(launch_cg_step<float, float>(dl, rin, p, w, K, P->slot(sa), P->slot(kPV), st), "cg step");
      dot_op<float, float>(P, rin, rin, K, kRR);
      double h[2];
      P->read_slots(kPV, 2, h);
      ++total;
      if (!std::isfinite(h[0]) || !std::isfinite(h[1]))
        throw Error{TS_EBREAKDOWN, "mixed CG breakdown: non-finite scalar"};
      report(every, "mixed", total, std::sqrt(h[1]));
      P->history.push_back(std::sqrt(h[1]));
      const bool breakdown = !(h[0] > 0.0);   // the device skipped the step
      if (breakdown && fresh) hip_check(launch_scale_copy<float, float>(p, dl, K, 1.0, nullptr, st), "copy");
      const double rn = std::sqrt(h[1]);
      if (breakdown || rn <= tol || rn <= delta * rmax || total >= P->opt.max_iter) {
        // reliable update: alpha += ||b|| dl in FP64, FP64 true residual
        hip_check(launch_axpy_conv<float, double>(dl, alpha, K, bnorm, nullptr, st), "update");
        hip_check(launch_fill<float>(dl, 0.0f, K, st), "fill");
        true_residual(P, alpha, b, r, v);
        dot_op<double, double>(P, r, r, K, kRR64);
        P->read_slots(kRR64, 1, &rr);
        ++updates;
        rel = std::sqrt(rr) / bnorm;
        P->history.back() = rel;
        if (!std::isfinite(rel)) throw Error{TS_EBREAKDOWN, "residual is not finite"};
        if (rel <= tol || total >= P->opt.max_iter || updates >= P->opt.max_refine) break;
        hip_check(launch_scale_copy<double, float>(r, rin, K, 1.0 / bnorm, nullptr, st), "to fp32");
        rmax = rel;
        if (breakdown) {   // restart the direction from the new residual
          run_captured(P, 3, capture_key(P, rin, z, nullptr), [&] { vcycle_op<float>(P, G, rin, z); });
          hip_check(launch_scale_copy<float, float>(z, p, K, 1.0, nullptr, st), "copy");
          dot_op<float, float>(P, rin, z, K, sa);
          fresh = true;
          continue;
        }
      }
      fresh = false;
      run_captured(P, 3, capture_key(P, rin, z, nullptr), [&] { vcycle_op<float>(P, G, rin, z); });
      dot_op<float, float>(P, rin, z, K, sb);
      hip_check(launch_p_update<float>(p, z, K, P->slot(sb), P->slot(sa), st), "p update");
      std::swap(sa, sb);
    }
  }
  info->iterations = total;
  info->refinements = updates;
  info->rel_residual = rel;
  info->converged = rel <= tol;
  return info->converged ? TS_OK : TS_ENOTCONV;
}

ts_status solve(Problem* P, double* alpha, int use_start, ts_solve_info* info_out) {
  auto t0 = std::chrono::steady_clock::now();
  ts_solve_info info{};
  const int64_t applies0 = P->applies;
  if (P->opt.preconditioner != TS_PC_MG && P->opt.precision != TS_FP64)
    throw Error{TS_EINVAL, "the mixed-precision modes run the V-cycle preconditioner (TS_PC_MG)"};
  P->history.clear();
  ts_status s;
  if (P->opt.precision == TS_FP64) s = solve_fp64(P, alpha, use_start, &info);
  else if (P->opt.precision == TS_MIXED_FP32_VCYCLE) s = solve_fp64(P, alpha, use_start, &info, true);
  else s = solve_mixed(P, alpha, use_start, &info);
  hip_check(hipStreamSynchronize(P->stream), "sync");
  info.setup_s = P->setup_s;
  info.solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  info.applies = P->applies - applies0;
  info.residual_history = P->history.data();
  info.history_len = int(P->history.size());
  if (info_out) *info_out = info;
  return s;
}

}  // namespace tsmg
