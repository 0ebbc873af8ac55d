// The extern "C" boundary declared in include/tsmg.h: argument checks,
// translation of internal errors into ts_status codes and the thread-local
// error message. No exception crosses this file.
#include <hip/hip_runtime.h>

#include <cstring>
#include <exception>
#include <string>

#include "api_util.h"
#include "problem.h"

namespace tsmg {
extern thread_local std::string g_last_error;
void rhs_op(Problem* P, double* b);
}  // namespace tsmg

using tsmg::Error;
using tsmg::Problem;

namespace {

Problem* get(const ts_problem* p) {
  if (!p || !p->impl) throw Error{TS_EINVAL, "null problem handle"};
  tsmg::hip_check(hipSetDevice(p->impl->device), "hipSetDevice");
  return p->impl;
}

void need(bool ok, const char* msg) {
  if (!ok) throw Error{TS_EINVAL, msg};
}

void check_level(const Problem* P, int level, int lo) {
  if (level < lo || level > P->G)
    throw Error{TS_EINVAL, "level " + std::to_string(level) + " outside " + std::to_string(lo) + ".." +
                               std::to_string(P->G)};
}

}  // namespace

extern "C" {

void ts_default_options(ts_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nu1 = 1;
  o->nu2 = 1;
  o->omega_scale = 1.8;
  o->lanczos_steps = 16;
  o->omega_fixed = 0.0;
  o->precision = TS_FP64;
  o->max_iter = 10000;
  o->tol = 1e-8;
  o->inner_tol = 0.1;
  o->max_refine = 50;
  o->points_per_block = 0;
  o->stencil_mode = 0;
  o->stream = nullptr;
  o->preconditioner = TS_PC_MG;
  o->smoother = TS_SMOOTH_JACOBI;
  o->ssor_omega = 1.0;
  o->coarse_solver = TS_COARSE_DIRECT;
  o->coarse_tol = 1e-14;
  o->coarse_max_iter = 20000;
  o->coarsest_level = 1;
}

const char* ts_version(void) { return "tsmg 0.1 gfx950"; }

const char* ts_last_error(void) { return tsmg::g_last_error.c_str(); }

ts_status ts_create(int d, int q, const int32_t* intervals, const double* lo, const double* hi, int64_t n,
                    const double* x, const double* y, double lambda, const ts_options* opt, ts_problem** out) {
  TS_API_BEGIN
  need(out != nullptr, "out must not be null");
  *out = nullptr;
  Problem* P = tsmg::create_problem(d, q, intervals, lo, hi, n, x, y, lambda, opt);
  *out = new ts_problem{P};
  return TS_OK;
  TS_API_END
}

void ts_destroy(ts_problem* p) {
  if (!p) return;
  try {
    if (p->impl) {
      (void)hipSetDevice(p->impl->device);
      delete p->impl;
    }
  } catch (...) {
  }
  delete p;
}

ts_status ts_set_options(ts_problem* p, const ts_options* opt) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(opt != nullptr, "opt must not be null");
  tsmg::check_solve_options(*opt);
  P->opt.preconditioner = opt->preconditioner;
  P->opt.smoother = opt->smoother;
  P->opt.ssor_omega = opt->ssor_omega;
  P->opt.coarse_tol = opt->coarse_tol;
  P->opt.coarse_max_iter = opt->coarse_max_iter;
  P->opt.nu1 = opt->nu1;
  P->opt.nu2 = opt->nu2;
  P->opt.precision = opt->precision;
  P->opt.max_iter = opt->max_iter;
  P->opt.tol = opt->tol;
  P->opt.inner_tol = opt->inner_tol;
  P->opt.max_refine = opt->max_refine;
  P->opt.vcycle_graph = opt->vcycle_graph;
  return TS_OK;
  TS_API_END
}

ts_status ts_bottom_level(const ts_problem* p, int* level) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(level != nullptr, "level must not be null");
  *level = tsmg::bottom_level(P);
  return TS_OK;
  TS_API_END
}

ts_status ts_num_levels(const ts_problem* p, int* G) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(G != nullptr, "G must not be null");
  *G = P->G;
  return TS_OK;
  TS_API_END
}

ts_status ts_num_coeffs(const ts_problem* p, int level, int64_t* K) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(K != nullptr, "K must not be null");
  check_level(P, level, 1);
  *K = P->lev[level].K;
  return TS_OK;
  TS_API_END
}

ts_status ts_get_omega(const ts_problem* p, int level, double* omega) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(omega != nullptr, "omega must not be null");
  check_level(P, level, 1);
  *omega = (level <= P->Gc) ? 0.0 : P->lev[level].omega;
  return TS_OK;
  TS_API_END
}

ts_status ts_rhs(ts_problem* p, double* b) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(b != nullptr, "b must not be null");
  tsmg::rhs_op(P, b);
  return TS_OK;
  TS_API_END
}

ts_status ts_apply(ts_problem* p, int level, const double* c, double* out) {
  TS_API_BEGIN
  Problem* P = get(p);
  check_level(P, level, P->Gc);
  need(c && out, "c and out must not be null");
  need(static_cast<const void*>(c) != static_cast<const void*>(out), "c and out must not alias");
  tsmg::apply_op<double>(P, level, c, out);
  return TS_OK;
  TS_API_END
}

ts_status ts_apply_f32(ts_problem* p, int level, const float* c, float* out) {
  TS_API_BEGIN
  Problem* P = get(p);
  check_level(P, level, P->Gc);
  need(c && out, "c and out must not be null");
  need(static_cast<const void*>(c) != static_cast<const void*>(out), "c and out must not alias");
  tsmg::apply_op<float>(P, level, c, out);
  return TS_OK;
  TS_API_END
}

ts_status ts_diag(ts_problem* p, int level, double* D) {
  TS_API_BEGIN
  Problem* P = get(p);
  check_level(P, level, P->Gc);
  need(D != nullptr, "D must not be null");
  const tsmg::Level& L = P->lev[level];
  tsmg::hip_check(hipMemcpyAsync(D, L.diag.p, sizeof(double) * L.K, hipMemcpyDeviceToDevice, P->stream),
                  "copy diag");
  return TS_OK;
  TS_API_END
}

ts_status ts_prolong(ts_problem* p, int level, const double* e, double* out) {
  TS_API_BEGIN
  Problem* P = get(p);
  check_level(P, level, P->Gc + 1);
  need(e && out, "e and out must not be null");
  tsmg::prolong_op<double>(P, level, e, out, false);
  return TS_OK;
  TS_API_END
}

ts_status ts_restrict(ts_problem* p, int level, const double* r, double* out) {
  TS_API_BEGIN
  Problem* P = get(p);
  check_level(P, level, P->Gc + 1);
  need(r && out, "r and out must not be null");
  tsmg::restrict_op<double>(P, level, r, out, static_cast<const double*>(nullptr));
  return TS_OK;
  TS_API_END
}

ts_status ts_coarse_solve(ts_problem* p, const double* b, double* x) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(b && x, "b and x must not be null");
  need(static_cast<const void*>(b) != static_cast<const void*>(x), "b and x must not alias");
  tsmg::coarse_op<double>(P, b, x);
  return TS_OK;
  TS_API_END
}

ts_status ts_vcycle(ts_problem* p, const double* r, double* z) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(r && z, "r and z must not be null");
  need(static_cast<const void*>(r) != static_cast<const void*>(z), "r and z must not alias");
  tsmg::vcycle_op<double>(P, P->G, r, z);
  return TS_OK;
  TS_API_END
}

ts_status ts_vcycle_f32(ts_problem* p, const float* r, float* z) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(r && z, "r and z must not be null");
  need(static_cast<const void*>(r) != static_cast<const void*>(z), "r and z must not alias");
  tsmg::vcycle_op<float>(P, P->G, r, z);
  return TS_OK;
  TS_API_END
}

ts_status ts_solve(ts_problem* p, double* alpha, int use_start, ts_solve_info* info) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(alpha != nullptr, "alpha must not be null");
  return tsmg::solve(P, alpha, use_start, info);
  TS_API_END
}

ts_status ts_evaluate(ts_problem* p, const double* alpha, int64_t m, const double* xq, double* yq) {
  TS_API_BEGIN
  Problem* P = get(p);
  need(m >= 0, "m must be >= 0");
  if (m == 0) return TS_OK;
  need(alpha && xq && yq, "alpha, xq and yq must not be null");
  if (P->general) tsmg::eval_general(P, alpha, m, xq, yq);
  else tsmg::hip_check(tsmg::launch_eval(P->d, alpha, xq, m, P->box, yq, P->stream), "evaluate");
  tsmg::hip_check(hipStreamSynchronize(P->stream), "sync");
  return TS_OK;
  TS_API_END
}

ts_status ts_profile_apply(ts_problem* p, int level, int fp32, int reps, double* ms_lambda, double* ms_data) {
  TS_API_BEGIN
  Problem* P = get(p);
  check_level(P, level, 1);
  need(reps >= 1, "reps must be >= 1");
  need(ms_lambda && ms_data, "outputs must not be null");
  if (fp32) tsmg::profile_apply<float>(P, level, reps, ms_lambda, ms_data);
  else tsmg::profile_apply<double>(P, level, reps, ms_lambda, ms_data);
  return TS_OK;
  TS_API_END
}

ts_status ts_memory(const ts_problem* p, size_t* resident, size_t* peak) {
  TS_API_BEGIN
  Problem* P = get(p);
  if (resident) *resident = size_t(P->mem_resident);
  if (peak) *peak = size_t(P->mem_peak);
  return TS_OK;
  TS_API_END
}

ts_status ts_footprint(int d, int q, const int32_t* intervals, int64_t n, const ts_options* opt,
                       size_t* bytes) {
  TS_API_BEGIN
  need(bytes != nullptr, "bytes must not be null");
  need(d >= 1 && d <= tsmg::kMaxDim, "d must be in 1..5");
  need(intervals != nullptr && n >= 1, "intervals must not be null and n >= 1");
  ts_options o;
  ts_default_options(&o);
  if (opt) o = *opt;
  for (int p = 0; p < d; ++p) need(intervals[p] >= 1, "intervals must be >= 1");
  if (tsmg::needs_general(d, q, intervals, o.degrees)) {
    *bytes = size_t(tsmg::footprint_general(d, q, intervals, n, o));
    return TS_OK;
  }
  const int N = intervals[0];
  *bytes = size_t(tsmg::footprint_bytes(d, N, n, o, 0.0));
  return TS_OK;
  TS_API_END
}

}  // extern "C"
