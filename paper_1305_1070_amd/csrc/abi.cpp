// C ABI of the library (declared in include/ndnegf.h): argument checking,
// error reporting, and the symbolic-analysis entry points.  The plan and
// solve entry points forward to the runtime (runtime.cpp).
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ndnegf.h"
#include "runtime.hpp"
#include "tree.hpp"

struct ndg_symbolic {
  ndg::Symbolic sy;
  ndg::OpCounts ops;
  double rgf_equiv = 0;
};

namespace {
thread_local std::string g_err;
}

namespace ndg {
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace ndg

using ndg::set_error;

static void fill_info(const ndg::Symbolic& sy, const ndg::OpCounts& oc, double rgf, int64_t ws,
                      ndg_info* out) {
  std::memset(out, 0, sizeof(*out));
  out->n = sy.n;
  out->nclusters = sy.nclusters;
  out->max_height = sy.max_height;
  out->max_cluster = sy.max_cluster;
  out->max_boundary = sy.max_boundary;
  out->ncontacts = (int32_t)sy.contact_cluster.size();
  out->nnz_boundary = (int64_t)sy.bidx.size();
  out->ops_fold_inv = oc.fold_inv;
  out->ops_fold_psi = oc.fold_psi;
  out->ops_fold_update = oc.fold_update;
  out->ops_gr_off = oc.gr_off;
  out->ops_gr_diag = oc.gr_diag;
  out->ops_gl_chain = oc.gl_chain;
  out->ops_gl_off = oc.gl_off;
  out->ops_gl_diag = oc.gl_diag;
  out->ops_total = oc.total();
  out->ops_rgf_equiv = rgf;
  out->workspace_bytes_per_energy = ws;
}

extern "C" {

ndg_status ndg_analyze(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                       int32_t ncontacts, const int32_t* const* contact_sites,
                       const int32_t* contact_n, const double* coords,
                       const ndg_tree_opts* opts, ndg_symbolic** out) {
  if (!out) { set_error("ndg_analyze: out is NULL"); return NDG_EINVAL; }
  *out = nullptr;
  if (ncontacts < 0 || (ncontacts > 0 && (!contact_sites || !contact_n))) {
    set_error("ndg_analyze: bad contact arguments");
    return NDG_EINVAL;
  }
  ndg::TreeOptions to;
  if (opts) {
    if (opts->leaf_max > 0) to.leaf_max = opts->leaf_max;
    if (opts->max_cluster > 0) to.max_cluster = opts->max_cluster;
    to.kind = opts->tree_kind;
    if (to.kind == 3) to.slab = opts->slab > 0 ? opts->slab : opts->slab == 0 ? 8 : 0;
    to.layer_of = opts->layer_of;
    if (opts->layer_max > ndg::kMaxCluster) {
      set_error("ndg_analyze: layer_max exceeds the kernels' limit of 128");
      return NDG_EINVAL;
    }
    to.layer_max = opts->layer_max > 0 ? opts->layer_max : ndg::kMaxCluster;
  } else {
    to.layer_max = ndg::kMaxCluster;
  }
  if (to.max_cluster > ndg::kMaxCluster) {
    set_error("ndg_analyze: max_cluster exceeds the kernels' limit of 128");
    return NDG_EINVAL;
  }
  auto* h = new (std::nothrow) ndg_symbolic;
  if (!h) { set_error("ndg_analyze: out of host memory"); return NDG_ENOMEM; }
  std::string err;
  int rc = ndg::build_symbolic(n, rowptr, col, val, ncontacts, contact_sites, contact_n, coords,
                               to, h->sy, err);
  if (rc != ndg::TREE_OK) {
    delete h;
    set_error("ndg_analyze: " + err);
    return rc == ndg::TREE_ENOTSYM ? NDG_ENOTSYM : rc == ndg::TREE_ECONTACT ? NDG_ECONTACT : NDG_EINVAL;
  }
  h->ops = ndg::count_ops(h->sy, true);
  // RGF comparison for layered devices: layers = distinct transport coordinates
  h->rgf_equiv = 0;
  if (coords) {
    int64_t nl = 0;
    double last = -1e300;
    std::vector<double> xs(n);
    for (int64_t i = 0; i < n; ++i) xs[i] = coords[3 * i];
    std::sort(xs.begin(), xs.end());
    for (double x : xs)
      if (x > last + 1e-9) { ++nl; last = x; }
    if (nl > 0 && n % nl == 0) h->rgf_equiv = ndg::rgf_ops(n / nl, nl);
  }
  *out = h;
  return NDG_OK;
}

void ndg_symbolic_destroy(ndg_symbolic* sy) { delete sy; }

ndg_status ndg_symbolic_costs(const ndg_symbolic* sy, int32_t capacity, ndg_kernel_stat* out,
                              int32_t* count) {
  if (!sy || !out || !count || capacity < 0) { set_error("ndg_symbolic_costs: bad argument"); return NDG_EINVAL; }
  const int rc = ndg::symbolic_costs(sy->sy, capacity, out, count);
  if (rc) set_error("ndg_symbolic_costs: capacity too small");
  return (ndg_status)rc;
}

ndg_status ndg_symbolic_info(const ndg_symbolic* sy, ndg_info* out) {
  if (!sy || !out) { set_error("ndg_symbolic_info: NULL argument"); return NDG_EINVAL; }
  fill_info(sy->sy, sy->ops, sy->rgf_equiv, ndg::workspace_bytes_per_energy(sy->sy), out);
  return NDG_OK;
}

ndg_status ndg_symbolic_arrays(const ndg_symbolic* h, int32_t* perm, int32_t* cl_off,
                               int32_t* parent, int32_t* height, int64_t* bptr, int32_t* bidx) {
  if (!h) { set_error("ndg_symbolic_arrays: NULL symbolic"); return NDG_EINVAL; }
  const auto& sy = h->sy;
  if (perm) std::memcpy(perm, sy.perm.data(), sizeof(int32_t) * sy.perm.size());
  if (cl_off) std::memcpy(cl_off, sy.cl_off.data(), sizeof(int32_t) * sy.cl_off.size());
  if (parent) std::memcpy(parent, sy.parent.data(), sizeof(int32_t) * sy.parent.size());
  if (height) std::memcpy(height, sy.height.data(), sizeof(int32_t) * sy.height.size());
  if (bptr) std::memcpy(bptr, sy.bptr.data(), sizeof(int64_t) * sy.bptr.size());
  if (bidx) std::memcpy(bidx, sy.bidx.data(), sizeof(int32_t) * sy.bidx.size());
  return NDG_OK;
}

ndg_status ndg_plan_create(const ndg_symbolic* sy, int32_t max_batch, int32_t device,
                           ndg_plan** out) {
  if (!sy || !out || max_batch <= 0) { set_error("ndg_plan_create: bad argument"); return NDG_EINVAL; }
  *out = nullptr;
  return (ndg_status)ndg::plan_create(sy->sy, sy->ops, max_batch, device, out);
}

ndg_status ndg_plan_destroy(ndg_plan* plan) { return (ndg_status)ndg::plan_destroy(plan); }

ndg_status ndg_plan_info(const ndg_plan* plan, ndg_info* out) {
  if (!plan || !out) { set_error("ndg_plan_info: NULL argument"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_info(plan, out);
}

ndg_status ndg_solve(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                     const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                     ndg_c128* diag_gr, ndg_c128* diag_gless, ndg_c128* diag_ggreater,
                     double* growth, ndg_precision prec, void* stream) {
  if (!plan) { set_error("ndg_solve: NULL plan"); return NDG_EINVAL; }
  if (nE < 0 || !(eta >= 0)) { set_error("ndg_solve: nE < 0 or eta < 0"); return NDG_EINVAL; }
  if (nE == 0) return NDG_OK;
  if (!E || !diag_gr || !diag_gless) { set_error("ndg_solve: NULL energy or output pointer"); return NDG_EINVAL; }
  if (prec != NDG_FP64 && prec != NDG_MIXED) { set_error("ndg_solve: unknown precision"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_solve(plan, nE, E, eta, V, sig_r, sig_less, diag_gr, diag_gless,
                                     diag_ggreater, growth, (int)prec, stream);
}

ndg_status ndg_solve_transport(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                               const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                               ndg_c128* diag_gr, ndg_c128* diag_gless, ndg_c128* diag_ggreater,
                               double* transmission, double* growth, void* stream) {
  if (!plan) { set_error("ndg_solve_transport: NULL plan"); return NDG_EINVAL; }
  if (nE < 0 || !(eta >= 0)) { set_error("ndg_solve_transport: nE < 0 or eta < 0"); return NDG_EINVAL; }
  if (nE == 0) return NDG_OK;
  if (!E || !diag_gr || !diag_gless) {
    set_error("ndg_solve_transport: NULL energy or output pointer");
    return NDG_EINVAL;
  }
  return (ndg_status)ndg::plan_run(plan, ndg::kRunSolve, nE, E, eta, V, sig_r, sig_less, diag_gr, diag_gless,
                                   nullptr, growth, nullptr, nullptr, nullptr, nullptr, NDG_FP64, stream,
                                   nullptr, nullptr, nullptr, nullptr, false, nullptr, 0, diag_ggreater,
                                   transmission);
}

ndg_status ndg_plan_enable_scattering(ndg_plan* plan) {
  if (!plan) { set_error("ndg_plan_enable_scattering: NULL plan"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_enable_scattering(plan);
}

ndg_status ndg_solve_scattering(ndg_plan* plan, int32_t nE, const double* E, double eta,
                                const double* V, const ndg_c128* const* sig_r,
                                const ndg_c128* const* sig_less, const ndg_c128* sig_r_ph,
                                const ndg_c128* sig_less_ph, ndg_c128* diag_gr, ndg_c128* diag_gless,
                                ndg_c128* diag_ggreater, double* growth, double* current, void* stream) {
  if (!plan) { set_error("ndg_solve_scattering: NULL plan"); return NDG_EINVAL; }
  if (nE < 0 || !(eta >= 0)) { set_error("ndg_solve_scattering: nE < 0 or eta < 0"); return NDG_EINVAL; }
  if (nE == 0) return NDG_OK;
  if (!E || !diag_gr || !diag_gless) {
    set_error("ndg_solve_scattering: NULL energy or output pointer");
    return NDG_EINVAL;
  }
  return (ndg_status)ndg::plan_run(plan, ndg::kRunSolve, nE, E, eta, V, sig_r, sig_less, diag_gr,
                                   diag_gless, diag_ggreater, growth, nullptr, nullptr, nullptr, nullptr,
                                   (int)NDG_FP64, stream, nullptr, sig_r_ph, sig_less_ph, current);
}

ndg_status ndg_scba(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                    const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, double d0, double mix,
                    double tol, int32_t max_iter, ndg_c128* sig_r_ph, ndg_c128* sig_less_ph,
                    ndg_c128* diag_gr, ndg_c128* diag_gless, ndg_c128* diag_ggreater, double* current,
                    int32_t* iterations, double* residual, void* stream) {
  if (!plan) { set_error("ndg_scba: NULL plan"); return NDG_EINVAL; }
  if (nE < 0 || !(eta >= 0) || !(d0 >= 0) || !(mix > 0 && mix <= 1) || !(tol >= 0) || max_iter < 1) {
    set_error("ndg_scba: nE < 0, eta < 0, d0 < 0, mix outside (0, 1], tol < 0 or max_iter < 1");
    return NDG_EINVAL;
  }
  if (nE == 0) {
    if (iterations) *iterations = 0;
    if (residual) *residual = 0.0;
    return NDG_OK;
  }
  if (!E || !sig_r_ph || !sig_less_ph || !diag_gr || !diag_gless) {
    set_error("ndg_scba: NULL energy, self-energy or output pointer");
    return NDG_EINVAL;
  }
  return (ndg_status)ndg::plan_scba(plan, nE, E, eta, V, sig_r, sig_less, d0, mix, tol, max_iter, sig_r_ph,
                                    sig_less_ph, diag_gr, diag_gless, diag_ggreater, current, iterations,
                                    residual, stream);
}

ndg_status ndg_poisson_newton_step(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                                   const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                                   const double* cE, const int64_t* k_rowptr, const int32_t* k_col,
                                   const double* k_val, int64_t k_nnz, double beta, const double* nd,
                                   double cg_tol, int32_t cg_max_iter, double* delta, double* res_norm,
                                   int32_t* cg_iterations, double* cg_residual, void* stream) {
  if (!plan) { set_error("ndg_poisson_newton_step: NULL plan"); return NDG_EINVAL; }
  if (nE < 0 || !(eta >= 0) || !(cg_tol >= 0) || cg_max_iter < 0 || k_nnz < 0) {
    set_error("ndg_poisson_newton_step: nE < 0, eta < 0, cg_tol < 0 or cg_max_iter < 0");
    return NDG_EINVAL;
  }
  if (!E || !V || !cE || !k_rowptr || !k_col || !k_val || !nd || !delta) {
    set_error("ndg_poisson_newton_step: NULL argument");
    return NDG_EINVAL;
  }
  return (ndg_status)ndg::plan_poisson_newton(plan, nE, E, eta, V, sig_r, sig_less, cE, k_rowptr, k_col, k_val,
                                              k_nnz, beta, nd, cg_tol, cg_max_iter, delta, res_norm, cg_iterations,
                                              cg_residual, stream);
}

static ndg_status check_common(const char* who, ndg_plan* plan, int32_t nE, const double* E, double eta,
                               ndg_precision prec) {
  if (!plan) { set_error(std::string(who) + ": NULL plan"); return NDG_EINVAL; }
  if (nE < 0 || !(eta >= 0)) { set_error(std::string(who) + ": nE < 0 or eta < 0"); return NDG_EINVAL; }
  if (nE > 0 && !E) { set_error(std::string(who) + ": NULL energies"); return NDG_EINVAL; }
  if (prec != NDG_FP64 && prec != NDG_MIXED) { set_error(std::string(who) + ": unknown precision"); return NDG_EINVAL; }
  return NDG_OK;
}

ndg_status ndg_density(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                       const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                       const double* cE, double* density, ndg_precision prec, void* stream) {
  ndg_status st = check_common("ndg_density", plan, nE, E, eta, prec);
  if (st != NDG_OK) return st;
  if (!cE || !density) { set_error("ndg_density: NULL weights or output"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_run(plan, ndg::kRunDensity, nE, E, eta, V, sig_r, sig_less, nullptr,
                                   nullptr, nullptr, nullptr, cE, density, nullptr, nullptr,
                                   (int)prec, stream);
}

ndg_status ndg_plan_enable_adjoint(ndg_plan* plan) {
  if (!plan) { set_error("ndg_plan_enable_adjoint: NULL plan"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_enable_adjoint(plan);
}

ndg_status ndg_density_vjp(ndg_plan* plan, int32_t nE, const double* E, double eta, const double* V,
                           const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                           const double* cE, const double* nbar, double* vbar, ndg_precision prec,
                           void* stream) {
  ndg_status st = check_common("ndg_density_vjp", plan, nE, E, eta, prec);
  if (st != NDG_OK) return st;
  if (!cE || !nbar || !vbar) { set_error("ndg_density_vjp: NULL weights, cotangent or output"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_run(plan, ndg::kRunVjp, nE, E, eta, V, sig_r, sig_less, nullptr,
                                   nullptr, nullptr, nullptr, cE, nullptr, nbar, vbar, (int)prec,
                                   stream);
}

ndg_status ndg_density_vjp_noalloc(ndg_plan* plan, int32_t nE, const double* E, double eta,
                                   const double* V, const ndg_c128* const* sig_r,
                                   const ndg_c128* const* sig_less, const double* cE,
                                   const double* nbar, double* vbar, ndg_precision prec, void* stream) {
  ndg_status st = check_common("ndg_density_vjp_noalloc", plan, nE, E, eta, prec);
  if (st != NDG_OK) return st;
  if (!cE || !nbar || !vbar) {
    set_error("ndg_density_vjp_noalloc: NULL weights, cotangent or output");
    return NDG_EINVAL;
  }
  int64_t cap = 0;
  double* part = ndg::noalloc_scratch(ndg::plan_device(plan), &cap);
  if (!part) {
    set_error("ndg_density_vjp_noalloc: the static buffer's device address is not available");
    return NDG_EHIP;
  }
  return (ndg_status)ndg::plan_run(plan, ndg::kRunVjp, nE, E, eta, V, sig_r, sig_less, nullptr,
                                   nullptr, nullptr, nullptr, cE, nullptr, nbar, vbar, (int)prec,
                                   stream, nullptr, nullptr, nullptr, nullptr, false, part, cap);
}

ndg_status ndg_plan_status(ndg_plan* plan, int32_t* code, int32_t* energy, int32_t* cluster) {
  if (!plan || !code || !energy || !cluster) { set_error("ndg_plan_status: NULL argument"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_status(plan, code, energy, cluster);
}

ndg_status ndg_plan_export_block(ndg_plan* plan, int32_t which, int32_t energy, int32_t cluster,
                                 ndg_c128* out) {
  if (!plan || !out) { set_error("ndg_plan_export_block: NULL argument"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_export_block(plan, which, energy, cluster, out);
}

ndg_status ndg_plan_set_profiling(ndg_plan* plan, int32_t enable) {
  if (!plan) { set_error("ndg_plan_set_profiling: NULL plan"); return NDG_EINVAL; }
  if (enable < 0 || enable > 2) { set_error("ndg_plan_set_profiling: mode must be 0, 1 or 2"); return NDG_EINVAL; }
  return (ndg_status)ndg::plan_set_profiling(plan, enable);
}

ndg_status ndg_plan_profile(ndg_plan* plan, int32_t capacity, ndg_kernel_stat* out,
                            int32_t* count) {
  if (!plan || !count || capacity < 0 || (capacity > 0 && !out)) {
    set_error("ndg_plan_profile: bad argument");
    return NDG_EINVAL;
  }
  return (ndg_status)ndg::plan_profile(plan, capacity, out, count);
}

const char* ndg_status_string(int32_t s) {
  switch (s) {
    case NDG_OK: return "ok";
    case NDG_EINVAL: return "invalid argument";
    case NDG_ENOTSYM: return "H is not symmetric";
    case NDG_ECONTACT: return "contact cannot be kept inside one cluster";
    case NDG_ESINGULAR: return "singular pivot block";
    case NDG_ENOMEM: return "out of device memory";
    case NDG_EHIP: return "HIP runtime error";
    case NDG_ENONFINITE: return "non-finite value";
    case NDG_ENOTSPD: return "Newton Jacobian not positive definite";
    default: return "unknown status";
  }
}

const char* ndg_last_error(void) { return g_err.c_str(); }

}  // extern "C"
