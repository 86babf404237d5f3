// Runtime of the library: plan (device workspace and level schedule) and
// solve orchestration.  Host code; kernels live in kernels.hip.
#pragma once

#include <cstdint>
#include <string>

#include "../../include/ndnegf.h"
#include "tree.hpp"

namespace ndg {

constexpr int kMaxCluster = 128;  // largest cluster the pivot kernels hold on chip
constexpr int kMaxClusterAux = 64;  // largest cluster of the adjoint and scattering kernels
constexpr int kMaxContacts = 2;  // contacts handled by the chain kernels
constexpr int kCostClasses = 7;  // launch groups per kernel and height (size classes)

void set_error(const std::string& msg);

int64_t workspace_bytes_per_energy(const Symbolic& sy);
// algorithmic work per energy of each launch group (host only, no plan)
int symbolic_costs(const Symbolic& sy, int capacity, ndg_kernel_stat* out, int32_t* count);

int plan_create(const Symbolic& sy, const OpCounts& oc, int max_batch, int device, ndg_plan** out);
int plan_destroy(ndg_plan* plan);
int plan_info(const ndg_plan* plan, ndg_info* out);
int plan_solve(ndg_plan* plan, int nE, const double* E, double eta, const double* V,
               const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, ndg_c128* dgr,
               ndg_c128* dgl, ndg_c128* dgg, double* growth, int prec, void* stream);
enum RunMode { kRunSolve = 0, kRunDensity = 1, kRunVjp = 2 };
int plan_run(ndg_plan* p, int mode, int nE, const double* E, double eta, const double* V,
             const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, ndg_c128* dgr,
             ndg_c128* dgl, ndg_c128* dgg, double* growth, const double* cE, double* density,
             const double* nbar, double* vbar, int prec, void* stream,
             const int32_t* e0p = nullptr, const ndg_c128* sig_r_ph = nullptr,
             const ndg_c128* sig_less_ph = nullptr, double* current = nullptr, bool reuse_fold = false,
             double* vjp_part = nullptr, int64_t vjp_part_capacity = 0,
             ndg_c128* dgg_explicit = nullptr, double* transmission = nullptr);
// The no-allocation density VJP's partials: a file-scope device array, its
// address on `device` (looked up once per device) and its size in doubles.
double* noalloc_scratch(int device, int64_t* capacity);
// One batch of energies starting at the device-resident index *e0p (for a
// graph replayed over the energy range): the launches of a single batch of
// max_batch energies, slots at or beyond nE skipped; growth is not cleared.
int plan_solve_chunk(ndg_plan* plan, int nE, const double* E, double eta, const double* V,
                     const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                     ndg_c128* dgr, ndg_c128* dgl, ndg_c128* dgg, double* growth, int prec,
                     void* stream, const int32_t* e0p);
int plan_max_batch(const ndg_plan* plan);
int plan_enable_adjoint(ndg_plan* plan);
int plan_enable_scattering(ndg_plan* plan);
int plan_poisson_newton(ndg_plan* p, int nE, const double* E, double eta, const double* V,
                        const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, const double* cE,
                        const int64_t* k_rowptr, const int32_t* k_col, const double* k_val, int64_t k_nnz,
                        double beta, const double* nd, double cg_tol, int cg_max_iter, double* delta,
                        double* res_norm, int32_t* cg_iterations, double* cg_residual, void* stream);
int plan_scba(ndg_plan* p, int nE, const double* E, double eta, const double* V,
              const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, double d0, double mix,
              double tol, int max_iter, ndg_c128* sig_r_ph, ndg_c128* sig_less_ph, ndg_c128* dgr,
              ndg_c128* dgl, ndg_c128* dgg, double* current, int32_t* iterations, double* residual,
              void* stream);
int plan_ncontacts(const ndg_plan* plan);
int plan_device(const ndg_plan* plan);
bool plan_profiling(const ndg_plan* plan);
int plan_status(ndg_plan* plan, int32_t* code, int32_t* energy, int32_t* cluster);
int plan_set_profiling(ndg_plan* plan, int mode);
int plan_profile(ndg_plan* plan, int capacity, ndg_kernel_stat* out, int32_t* count);
int plan_export_block(ndg_plan* plan, int which, int energy, int cluster, ndg_c128* out);

}  // namespace ndg
