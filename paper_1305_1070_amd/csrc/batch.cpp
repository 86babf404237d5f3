// Batched solve of several devices in one captured graph.
//
// Energies and devices are independent problems (Section 3.2 processes one
// energy at a time), so a batch of uneven devices is a set of independent
// level-by-level launch sequences.  One batch of energies per device (the
// plan's max_batch) is captured into one HIP graph with a branch per device
// (fork/join through events on per-device capture streams); the first
// energy of each device's batch lives in device memory and a final node
// advances it, so replaying the same graph sweeps the whole energy range
// with each plan's workspace bounded by its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ndnegf.h"
#include "kernels.hpp"
#include "runtime.hpp"

struct ndg_batch {
  int device = -1;
  std::vector<ndg_plan*> plans;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  int32_t* d_e0 = nullptr;   // per plan: first energy of the current replay
  int32_t* d_inc = nullptr;  // per plan: its batch size
  int replays = 0;
  int launches = 0;          // graph launches of the last solve
  hipGraph_t graph = nullptr;      // one batch of energies of every plan
  hipGraph_t whole = nullptr;      // the counter resets, then `replays` copies of graph
  hipGraphExec_t exec = nullptr;   // of whole, or of graph when whole could not be built
  bool single = false;             // exec runs the whole energy range
  // the argument set the cached graph was captured with
  std::vector<ndg_solve_args> key;
  std::vector<std::vector<const ndg_c128*>> key_sig;
  int key_prec = -1;
};

namespace {

void release_graph(ndg_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->whole) (void)hipGraphDestroy(b->whole);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->whole = nullptr;
  b->graph = nullptr;
  b->single = false;
  b->key.clear();
  b->key_sig.clear();
  b->key_prec = -1;
}

bool same_key(const ndg_batch* b, const ndg_solve_args* args, int prec) {
  if (!b->exec || b->key_prec != prec || b->key.size() != b->plans.size()) return false;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const ndg_solve_args& a = args[i];
    const ndg_solve_args& k = b->key[i];
    if (a.nE != k.nE || a.E != k.E || a.eta != k.eta || a.V != k.V || a.diag_gr != k.diag_gr ||
        a.diag_gless != k.diag_gless || a.diag_ggreater != k.diag_ggreater || a.growth != k.growth)
      return false;
    const int nc = ndg::plan_ncontacts(b->plans[i]);
    for (int c = 0; c < nc; ++c)
      if (a.sig_r[c] != b->key_sig[i][2 * c] || a.sig_less[c] != b->key_sig[i][2 * c + 1]) return false;
  }
  return true;
}

}  // namespace

extern "C" {

ndg_status ndg_batch_create(int32_t nplans, ndg_plan* const* plans, ndg_batch** out) {
  if (!out || nplans <= 0 || !plans) { ndg::set_error("ndg_batch_create: bad argument"); return NDG_EINVAL; }
  *out = nullptr;
  for (int i = 0; i < nplans; ++i) {
    if (!plans[i]) { ndg::set_error("ndg_batch_create: NULL plan"); return NDG_EINVAL; }
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) { ndg::set_error("ndg_batch_create: a plan appears twice"); return NDG_EINVAL; }
  }
  auto* b = new (std::nothrow) ndg_batch;
  if (!b) { ndg::set_error("ndg_batch_create: out of host memory"); return NDG_ENOMEM; }
  b->plans.assign(plans, plans + nplans);
  const int dev = ndg::plan_device(plans[0]);
  for (int i = 1; i < nplans; ++i)
    if (ndg::plan_device(plans[i]) != dev) {
      delete b;
      ndg::set_error("ndg_batch_create: the plans must live on one device");
      return NDG_EINVAL;
    }
  b->device = dev;
  if (hipSetDevice(dev) != hipSuccess ||
      hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
    delete b;
    ndg::set_error("ndg_batch_create: HIP event creation failed");
    return NDG_EHIP;
  }
  std::vector<int32_t> inc(nplans);
  for (int i = 0; i < nplans; ++i) inc[i] = ndg::plan_max_batch(plans[i]);
  if (hipMalloc((void**)&b->d_e0, sizeof(int32_t) * nplans) != hipSuccess ||
      hipMalloc((void**)&b->d_inc, sizeof(int32_t) * nplans) != hipSuccess ||
      hipMemcpy(b->d_inc, inc.data(), sizeof(int32_t) * nplans, hipMemcpyHostToDevice) != hipSuccess) {
    ndg_batch_destroy(b);
    ndg::set_error("ndg_batch_create: device allocation failed");
    return NDG_ENOMEM;
  }
  for (int i = 0; i < nplans; ++i) {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    // default priority: every stream of the library uses the default
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      ndg_batch_destroy(b);
      ndg::set_error("ndg_batch_create: HIP stream creation failed");
      return NDG_EHIP;
    }
    b->streams.push_back(s);
    b->done.push_back(ev);
  }
  *out = b;
  return NDG_OK;
}

int32_t ndg_batch_launches(const ndg_batch* b) { return b ? b->launches : 0; }

ndg_status ndg_batch_destroy(ndg_batch* b) {
  if (!b) return NDG_OK;
  // replays still in flight read the graph and the offsets freed below
  if (b->device >= 0 && hipSetDevice(b->device) == hipSuccess) (void)hipDeviceSynchronize();
  release_graph(b);
  for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->d_e0) (void)hipFree(b->d_e0);
  if (b->d_inc) (void)hipFree(b->d_inc);
  delete b;
  return NDG_OK;
}

ndg_status ndg_batch_solve(ndg_batch* b, const ndg_solve_args* args, ndg_precision prec,
                           void* stream) {
  if (!b || !args) { ndg::set_error("ndg_batch_solve: NULL argument"); return NDG_EINVAL; }
  if (prec != NDG_FP64 && prec != NDG_MIXED) { ndg::set_error("ndg_batch_solve: unknown precision"); return NDG_EINVAL; }
  const int np = (int)b->plans.size();
  for (int i = 0; i < np; ++i) {
    const ndg_solve_args& a = args[i];
    if (a.nE <= 0 || !a.E || !a.diag_gr || !a.diag_gless || !(a.eta >= 0)) {
      ndg::set_error("ndg_batch_solve: bad arguments for device " + std::to_string(i));
      return NDG_EINVAL;
    }
    const int nc = ndg::plan_ncontacts(b->plans[i]);
    if (nc > 0 && (!a.sig_r || !a.sig_less)) { ndg::set_error("ndg_batch_solve: missing self-energies"); return NDG_EINVAL; }
    for (int c = 0; c < nc; ++c)
      if (!a.sig_r[c] || !a.sig_less[c]) { ndg::set_error("ndg_batch_solve: NULL self-energy"); return NDG_EINVAL; }
  }
  for (int i = 0; i < np; ++i)
    if (ndg::plan_profiling(b->plans[i])) {
      // per-launch timing events cannot be recorded into a graph
      ndg::set_error("ndg_batch_solve: switch profiling off on the batch's plans");
      return NDG_EINVAL;
    }
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(ndg::plan_device(b->plans[0])) != hipSuccess) { ndg::set_error("ndg_batch_solve: hipSetDevice failed"); return NDG_EHIP; }
  if (!same_key(b, args, (int)prec)) {
    release_graph(b);
    if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) {
      ndg::set_error("ndg_batch_solve: hipStreamBeginCapture failed");
      return NDG_EHIP;
    }
    int rc = NDG_OK;
    (void)hipEventRecord(b->fork, st);
    for (int i = 0; i < np && rc == NDG_OK; ++i) {
      (void)hipStreamWaitEvent(b->streams[i], b->fork, 0);
      const ndg_solve_args& a = args[i];
      rc = ndg::plan_solve_chunk(b->plans[i], a.nE, a.E, a.eta, a.V, a.sig_r, a.sig_less,
                                 a.diag_gr, a.diag_gless, a.diag_ggreater, a.growth, (int)prec,
                                 b->streams[i], b->d_e0 + i);
      (void)hipEventRecord(b->done[i], b->streams[i]);
      (void)hipStreamWaitEvent(st, b->done[i], 0);
    }
    if (rc == NDG_OK) ndg::launch_advance(b->d_e0, b->d_inc, np, st);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rc != NDG_OK) {
      if (g) (void)hipGraphDestroy(g);
      return (ndg_status)rc;
    }
    if (ec != hipSuccess || !g) { ndg::set_error("ndg_batch_solve: hipStreamEndCapture failed"); return NDG_EHIP; }
    b->graph = g;
    // The whole energy range as one graph: the resets of the first-energy
    // counters and growth outputs (captured kernels), then one child copy
    // of the batch graph per replay, in sequence.  If it cannot be built,
    // the batch graph is launched once per replay instead.
    int replays = 0;
    for (int i = 0; i < np; ++i) {
      const int mb = ndg::plan_max_batch(b->plans[i]);
      replays = std::max(replays, (args[i].nE + mb - 1) / mb);
    }
    hipGraph_t w = nullptr;
    bool whole_ok = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (whole_ok) {
      ndg::launch_fill_zero_i32(b->d_e0, np, st);
      for (int i = 0; i < np; ++i)
        if (args[i].growth) ndg::launch_fill_zero(args[i].growth, args[i].nE, st);
      whole_ok = hipStreamEndCapture(st, &w) == hipSuccess && w;
    }
    if (whole_ok) {
      hipGraphNode_t prev = nullptr, node = nullptr;
      // every reset node is a dependency of the first copy
      std::vector<hipGraphNode_t> all;
      size_t nall = 0;
      whole_ok = hipGraphGetNodes(w, nullptr, &nall) == hipSuccess && nall > 0;
      if (whole_ok) {
        all.resize(nall);
        whole_ok = hipGraphGetNodes(w, all.data(), &nall) == hipSuccess;
      }
      for (int r = 0; r < replays && whole_ok; ++r) {
        whole_ok = hipGraphAddChildGraphNode(&node, w, r ? &prev : all.data(), r ? 1 : all.size(), g) == hipSuccess;
        prev = node;
      }
    }
    hipGraphExec_t ex = nullptr;
    if (whole_ok && hipGraphInstantiate(&ex, w, nullptr, nullptr, 0) == hipSuccess) {
      b->whole = w;
      b->single = true;
    } else {
      (void)hipGetLastError();
      if (w) (void)hipGraphDestroy(w);
      ex = nullptr;
      if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        release_graph(b);
        ndg::set_error("ndg_batch_solve: hipGraphInstantiate failed");
        return NDG_EHIP;
      }
    }
    b->exec = ex;
    b->key.assign(args, args + np);
    b->key_sig.assign(np, {});
    for (int i = 0; i < np; ++i) {
      const int nc = ndg::plan_ncontacts(b->plans[i]);
      for (int c = 0; c < nc; ++c) {
        b->key_sig[i].push_back(args[i].sig_r[c]);
        b->key_sig[i].push_back(args[i].sig_less[c]);
      }
      // the host arrays of pointers need not outlive the call
      b->key[i].sig_r = nullptr;
      b->key[i].sig_less = nullptr;
    }
    b->key_prec = (int)prec;
  }
  // replays needed for the longest energy range
  int replays = 0;
  for (int i = 0; i < np; ++i) {
    const int mb = ndg::plan_max_batch(b->plans[i]);
    replays = std::max(replays, (args[i].nE + mb - 1) / mb);
  }
  if (b->single) {
    if (hipGraphLaunch(b->exec, st) != hipSuccess) {
      ndg::set_error("ndg_batch_solve: hipGraphLaunch failed");
      return NDG_EHIP;
    }
    b->launches = 1;
  } else {
    // the counters and the growth outputs cleared by kernels outside the graph
    ndg::launch_fill_zero_i32(b->d_e0, np, st);
    for (int i = 0; i < np; ++i)
      if (args[i].growth) ndg::launch_fill_zero(args[i].growth, args[i].nE, st);
    for (int r = 0; r < replays; ++r)
      if (hipGraphLaunch(b->exec, st) != hipSuccess) {
        ndg::set_error("ndg_batch_solve: hipGraphLaunch failed");
        return NDG_EHIP;
      }
    b->launches = replays;
  }
  b->replays = replays;
  return NDG_OK;
}

}  // extern "C"
