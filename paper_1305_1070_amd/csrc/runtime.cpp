// Plan creation (device workspace, level schedule) and solve orchestration.
//
// Per energy, the solve runs the three stages of Section 3.2 level by level:
//   fold      heights 1 .. L:   assemble fronts, invert pivot blocks, Psi,
//                               Schur contributions (and the forward solve
//                               along each contact's chain for G^<);
//   extract   heights L .. 1:   G^r off-diagonal and diagonal blocks, then the
//                               G^< source on the contact chains and the G^<
//                               blocks;
//   epilogue  diagonals in the caller's site order, G^> from G^< + G^r - G^r+.
// Clusters of one height are independent (rule 1 of Section 3.2), so every
// launch covers (energies in the batch) x (clusters or tiles of one height).
#include "runtime.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ndnegf.h"
#include "kernels.hpp"

struct ndg_plan {
  int device = 0;
  int max_batch = 0;
  int64_t n = 0;
  int nclusters = 0;
  int max_height = 0;
  int ncontacts = 0;
  int nc[2] = {0, 0};
  int64_t stride = 0;  // complex elements per energy slab
  ndg::OpCounts ops;
  ndg_info info{};
  std::vector<ndg::ClusterDesc> hdesc;
  std::vector<int32_t> hbidx;
  std::vector<int32_t> hdeg;   // children count (host)
  std::vector<int32_t> hheight;
  // device arrays
  ndg::ClusterDesc* d_cl = nullptr;
  int32_t *d_relmap = nullptr, *d_kids_ptr = nullptr, *d_kids = nullptr;
  int32_t *d_hrow = nullptr, *d_hcol = nullptr;
  double* d_hval = nullptr;
  int32_t *d_perm = nullptr, *d_owner = nullptr;
  int32_t* d_cpos[2] = {nullptr, nullptr};
  int32_t *d_srow = nullptr, *d_scol = nullptr, *d_scid = nullptr, *d_sflat = nullptr;
  double* d_hfront = nullptr;
  int32_t *d_smap = nullptr, *d_pinv = nullptr;
  int32_t* d_gaddr = nullptr;
  int32_t* d_caddr = nullptr;  // contact blocks' stored-entry offsets (terminal currents)
  double2* d_src[2] = {nullptr, nullptr};  // per-batch sources of the extra G^< passes
  ndg::SiteDiag* d_sdiag = nullptr;
  int32_t* d_levels = nullptr;       // clusters by height
  ndg::ColItem* d_colitems = nullptr;
  ndg::UpdItem* d_upditems = nullptr;
  ndg::ChainItem* d_chainitems = nullptr;
  int32_t* d_chaincls = nullptr;
  std::vector<int> lvl_ptr, col_ptr, upd_ptr, chain_ptr, chaincl_ptr;  // per height (1-based)
  // adjoint solves per height: dynamic LDS of the one-wavefront variant (0:
  // no such cluster) and whether a cluster needs the tiled one
  std::vector<size_t> rhs_lds_fwd, rhs_lds_back;
  std::vector<char> rhs_big;
  // per height, the clusters split into size classes: fronts f <= 32, f <= 64
  // (whole on chip), then larger fronts with s <= 16, s <= 32, s <= 64,
  // s <= 128 (separate kernels, tile height following s; 64-row tiles above)
  struct Group { int cl0 = 0, ncl = 0, col0 = 0, ncol = 0, upd0 = 0, nupd = 0, size = 0; size_t lds = 0, lds_leaf = 0; };
  static constexpr int kClasses = 7;
  std::vector<Group> groups;  // [(H + 1) * kClasses]
  double2* d_ws = nullptr;
  int32_t* d_status = nullptr;
  // adjoint workspace (ndg_plan_enable_adjoint): right-hand sides Y, solutions
  // X, contact columns of G, per-cluster front vectors, per-energy partials
  double2 *d_rX = nullptr, *d_rG = nullptr, *d_rZ = nullptr;
  int32_t* d_cinv = nullptr;  // internal position -> column among all contacts' columns, or -1
  int64_t* d_ovec = nullptr;
  int32_t* d_bidx = nullptr;
  double* d_part = nullptr;
  int64_t zstride = 0;
  int mmax = 0;
  // Newton step of the Schroedinger-Poisson problem (allocated with the
  // adjoint workspace): kPoissonVecs vectors of n doubles, dot-product scratch
  static constexpr int kPoissonVecs = 7;
  double* d_pvec = nullptr;
  double* d_pdot = nullptr;
  int contact_cl[2] = {-1, -1};
  // phonon G^< source (ndg_plan_enable_scattering): all-ancestor rows, per
  // height and tile class (clusters s <= 16, <= 32, <= 64) the column tiles
  // of the frames and the clusters
  ndg::ScatDesc* d_sd = nullptr;
  int32_t* d_atab = nullptr;
  ndg::BPos* d_bpos = nullptr;
  ndg::LkItem* d_lk = nullptr;
  int32_t* d_umap = nullptr;
  ndg::ColItem* d_ancitems = nullptr;
  int32_t* d_anccls = nullptr;
  double2* d_sws = nullptr;
  double* d_scba = nullptr;  // Born loop reduction scratch: kScbaBlocks x 2 partials, then 2 maxima
  int64_t sstride = 0;
  struct AncGroup { int it0 = 0, nit = 0, cl0 = 0, ncl = 0; };
  std::vector<AncGroup> anc_groups;  // [(H + 1) * 3]
  int last_batch = 0;
  // algorithmic work per energy of each launch group: kernel, height, size
  // class (tile class for the scattering kernels); cost_index()
  std::vector<double> cost_flops, cost_bytes;
  int profiling_mode = 0;  // 2: every launch on the caller's stream (no overlap)
  // profiling
  bool profiling = false;
  struct Rec { int kid, h, q; hipEvent_t a, b; double flops, bytes; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> event_pool;
  // the G^< extraction runs on a second stream, concurrent with the G^r
  // extraction; the chain back substitution it needs runs ahead of it on a
  // third, which marks each finished height with an event
  hipStream_t side = nullptr, chain = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<hipEvent_t> ev_chain;  // [H + 1]
};

namespace ndg {

namespace {

enum KernelId {
  K_ASSEMBLE, K_FACTOR, K_PSI, K_UPDATE, K_CHAIN_FWD, K_DOWN_OFF_G, K_DOWN_DIAG_G, K_CHAIN_BACK,
  K_DOWN_OFF_P, K_DOWN_DIAG_P, K_EPILOGUE, K_FOLD_SMALL, K_EXTRACT_SMALL, K_RHS_FWD, K_RHS_BACK,
  K_VJP, K_EXTRACT_SMALL_P, K_ANC_G, K_ANC_N, K_ANC_P0, K_CHAIN_T, kKernels
};
const char* const kKernelNames[kKernels] = {
    "k_assemble", "k_factor", "k_psi", "k_update", "k_chain_fwd", "k_down_off(G)",
    "k_down_diag(G)", "k_chain_back", "k_down_off(P)", "k_down_diag(P)", "k_epilogue",
    "k_fold_small", "k_extract_small(G)", "k_rhs_fwd", "k_rhs_back", "k_vjp",
    "k_extract_small(P)", "k_anc_g", "k_anc_n", "k_anc_p0", "k_chain_t"};

int64_t align8(int64_t x) { return (x + 7) & ~int64_t(7); }

// Lays out one energy slab; fills desc offsets.  Returns the slab size.
int64_t layout(const Symbolic& sy, std::vector<ClusterDesc>& desc) {
  const int nc = sy.nclusters;
  desc.assign(nc, ClusterDesc{});
  const int ncont = (int)sy.contact_cluster.size();
  std::vector<int32_t> mask(nc, 0), chain_child(2 * nc, -1);
  for (int c = 0; c < ncont && c < kMaxContacts; ++c) {
    int prev = -1;
    for (int k = sy.contact_cluster[c]; k >= 0; k = sy.parent[k]) {
      mask[k] |= 1 << c;
      chain_child[2 * k + c] = prev;
      prev = k;
    }
  }
  // the rows of the G^r fronts of all clusters first, then those of the G^<
  // fronts in the same arrangement: a G^< entry sits a fixed distance after
  // its G^r counterpart (one gather table serves both)
  int64_t off = 0;
  for (int k = 0; k < nc; ++k) {
    desc[k].o_fg = off;
    off = align8(off + (int64_t)sy.s(k) * (sy.s(k) + sy.b(k)));
  }
  const int64_t pdelta = off;
  for (int k = 0; k < nc; ++k) desc[k].o_fp = desc[k].o_fg + pdelta;
  off = 2 * pdelta;
  for (int k = 0; k < nc; ++k) {
    ClusterDesc& d = desc[k];
    d.s = sy.s(k);
    d.b = sy.b(k);
    d.f = d.s + d.b;
    d.parent = sy.parent[k];
    d.pt_off = sy.cl_off[k];
    d.bptr = (int32_t)sy.bptr[k];
    d.hptr0 = (int32_t)sy.hptr[k];
    d.hptr1 = (int32_t)sy.hptr[k + 1];
    d.sptr0 = (int32_t)sy.sptr[k];
    d.sptr1 = (int32_t)sy.sptr[k + 1];
    d.chain_mask = mask[k];
    d.nself = 0;
    if (d.parent >= 0)
      for (int64_t q = sy.bptr[k]; q < sy.bptr[k + 1] && sy.owner[sy.bidx[q]] == d.parent; ++q) d.nself++;
    const int64_t s = d.s, b = d.b, f = d.f;
    d.o_ainv = off; off = align8(off + s * s);
    d.o_psi = off;  off = align8(off + s * b);
    d.o_upd = off;  off = align8(off + b * b);
    for (int c = 0; c < 2; ++c) {
      d.chain_child[c] = chain_child[2 * k + c];
      d.o_zf[c] = d.o_xf[c] = d.o_t[c] = -1;
      if (c < ncont && ((mask[k] >> c) & 1)) {
        const int64_t sc = (int64_t)sy.contact_pos[c].size();
        d.o_zf[c] = off; off = align8(off + f * sc);
        d.o_xf[c] = off; off = align8(off + f * sc);
        d.o_t[c] = off;  off = align8(off + s * sc);
      }
    }
  }
  return off;
}

template <class T>
int upload(T** dst, const T* src, size_t count) {
  *dst = nullptr;
  if (count == 0) return 0;
  if (hipMalloc((void**)dst, sizeof(T) * count) != hipSuccess) return NDG_ENOMEM;
  if (hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice) != hipSuccess) return NDG_EHIP;
  return 0;
}

void free_plan(ndg_plan* p) {
  if (!p) return;
  void* ptrs[] = {p->d_cl,        p->d_relmap,   p->d_kids_ptr,   p->d_kids,       p->d_hrow,
                  p->d_hcol,      p->d_hval,     p->d_perm,       p->d_owner,      p->d_cpos[0],
                  p->d_cpos[1],   p->d_levels,   p->d_colitems,   p->d_upditems,   p->d_chainitems,
                  p->d_chaincls,  p->d_ws,       p->d_status,     p->d_cinv,       p->d_rX,
                  p->d_rG,        p->d_rZ,       p->d_ovec,       p->d_bidx,       p->d_part,
                  p->d_srow,      p->d_scol,     p->d_scid,       p->d_sflat,      p->d_hfront,
                  p->d_smap,      p->d_pinv,     p->d_gaddr,      p->d_sdiag,      p->d_sd,
                  p->d_atab,      p->d_bpos,     p->d_lk,         p->d_umap,       p->d_ancitems,
                  p->d_anccls,    p->d_sws,      p->d_scba,       p->d_caddr,      p->d_pvec,
                  p->d_src[0],    p->d_src[1],
                  p->d_pdot};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (auto& r : p->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t ev : p->event_pool) (void)hipEventDestroy(ev);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  for (hipEvent_t ev : p->ev_chain)
    if (ev) (void)hipEventDestroy(ev);
  if (p->side) (void)hipStreamDestroy(p->side);
  if (p->chain) (void)hipStreamDestroy(p->chain);
  delete p;
}

}  // namespace

// Size class of cluster k: fronts of at most 32, 48, 64 points (whole on
// chip), then larger fronts by cluster size s <= 16, 32, 64, 128.
int size_class(const Symbolic& sy, int k) {
  const int s_ = sy.s(k), f = s_ + sy.b(k);
  if (f <= 32) return 0;
  if (f <= 48) return 1;
  if (f <= kSmallFront) return 2;
  return s_ <= 16 ? 3 : s_ <= 32 ? 4 : s_ <= 64 ? 5 : 6;
}

int cost_index(int kid, int h, int q, int H) { return (kid * (H + 1) + h) * kCostClasses + q; }

// Algorithmic work per energy of every launch group of the phonon-free solve
// (kernel, height, size class), in Section 4.1's convention: a product of
// i x j by j x k counts ijk complex multiply-adds, an i x i inversion i^3,
// 8 real flops each; bytes count each input block read once and each output
// block written once (16 per complex entry), a symmetric block (a Schur
// contribution, X_BB) by its distinct entries b (b + 1) / 2.  The flops of
// all groups sum to 8 times count_ops' total.
void phonon_free_costs(const Symbolic& sy, const std::vector<ClusterDesc>& hd, const int* nc_contact,
                       int ncontacts, std::vector<double>& fl, std::vector<double>& by) {
  const int nc = sy.nclusters, H = sy.max_height;
  fl.assign((size_t)kKernels * (H + 1) * kCostClasses, 0.0);
  by.assign(fl.size(), 0.0);
  auto addc = [&](int kid, int h, int q, double f_, double b_) {
    fl[cost_index(kid, h, q, H)] += f_;
    by[cost_index(kid, h, q, H)] += b_;
  };
  for (int k = 0; k < nc; ++k) {
    const int h = sy.height[k], q = size_class(sy, k);
    const double s = sy.s(k), b = sy.b(k), f = s + b;
    const bool leaf = sy.children[k].empty();
    // the children's contributions, symmetric: their distinct entries
    double kidb = 0;
    for (int32_t ch : sy.children[k]) kidb += (double)sy.b(ch) * (sy.b(ch) + 1) / 2;
    if (s + b <= kSmallFront) {
      // pivot inverse, Psi and the Schur contribution of the whole front
      addc(K_FOLD_SMALL, h, q, 8.0 * (s * s * s + s * s * b + s * b * b),
           16.0 * (kidb + s * s + s * b + b * (b + 1) / 2));
      // X_BB counted by its distinct entries (symmetric for G^r,
      // anti-Hermitian for G^<): b (b + 1) / 2.  A leaf off the contact
      // chains forms the diagonal of X_ii only.
      const bool diag_only = leaf && hd[k].chain_mask == 0;
      for (int kid : {K_EXTRACT_SMALL, K_EXTRACT_SMALL_P})
        addc(kid, h, q, 8.0 * (s * b * b + (diag_only ? s * b : s * s * b)),
             16.0 * (b * (b + 1) / 2 + s * s + s * b) + 16.0 * (diag_only ? s : s * b + s * s));
    } else {
      // the cluster's rows written once, each child's contribution to them
      // (its first nself boundary rows) read once
      double kidrows = 0;
      for (int32_t ch : sy.children[k]) kidrows += (double)hd[ch].nself * sy.b(ch);
      addc(K_ASSEMBLE, h, q, 0.0, 16.0 * (s * f + kidrows));
      addc(K_FACTOR, h, q, 8.0 * s * s * s, 16.0 * 2 * s * s);
      addc(K_PSI, h, q, 8.0 * s * s * b, 16.0 * (s * s + 2 * s * b));
      // F_BB gathered and U written by their distinct entries
      addc(K_UPDATE, h, q, 8.0 * s * b * b, 16.0 * (2 * s * b + b * (b + 1)));
      for (int kid : {K_DOWN_OFF_G, K_DOWN_OFF_P})
        addc(kid, h, q, 8.0 * s * b * b, 16.0 * (s * b + b * (b + 1) / 2 + s * b));
      for (int kid : {K_DOWN_DIAG_G, K_DOWN_DIAG_P}) addc(kid, h, q, 8.0 * s * s * b, 16.0 * (2 * s * b + 2 * s * s));
    }
    // the contact chains launch once per height (class 0)
    for (int c = 0; c < ncontacts; ++c) {
      if (!((hd[k].chain_mask >> c) & 1)) continue;
      const double sc = nc_contact[c];
      addc(K_CHAIN_FWD, h, 0, 8.0 * (s * b * sc + s * s * sc), 16.0 * (s * b + s * s + 2 * f * sc));
      addc(K_CHAIN_BACK, h, 0, 8.0 * (s * b * sc + s * sc * f), 16.0 * (s * b + 3 * f * sc + s * sc + s * f));
      // T = Zd Sigma^<: one launch for all chain clusters, after the fold
      addc(K_CHAIN_T, 0, 0, 8.0 * s * sc * sc, 16.0 * (2 * s * sc + sc * sc));
    }
  }
  addc(K_EPILOGUE, 0, 0, 0.0, 16.0 * 5.0 * (double)sy.n);
}

int64_t workspace_bytes_per_energy(const Symbolic& sy) {
  std::vector<ClusterDesc> desc;
  return layout(sy, desc) * 16;
}

int plan_create(const Symbolic& sy, const OpCounts& oc, int max_batch, int device, ndg_plan** out) {
  if ((int)sy.contact_cluster.size() > kMaxContacts) {
    set_error("ndg_plan_create: at most 2 contacts are supported");
    return NDG_EINVAL;
  }
  if (sy.max_cluster > kMaxCluster) {  // (contacts larger than this span a chain)
    set_error("ndg_plan_create: a cluster exceeds 128 points");
    return NDG_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    set_error("ndg_plan_create: no such HIP device");
    return NDG_EHIP;
  }
  if (hipSetDevice(device) != hipSuccess) { set_error("ndg_plan_create: hipSetDevice failed"); return NDG_EHIP; }
  auto* p = new ndg_plan;
  p->device = device;
  p->max_batch = max_batch;
  p->n = sy.n;
  p->nclusters = sy.nclusters;
  p->max_height = sy.max_height;
  p->ncontacts = (int)sy.contact_cluster.size();
  for (int c = 0; c < p->ncontacts; ++c) p->nc[c] = (int)sy.contact_pos[c].size();
  p->ops = oc;
  p->stride = layout(sy, p->hdesc);
  p->hbidx = sy.bidx;
  p->hheight = sy.height;
  for (int c = 0; c < p->ncontacts && c < 2; ++c) p->contact_cl[c] = sy.contact_cluster[c];
  const int nc = sy.nclusters, H = sy.max_height;
  // schedules per height
  std::vector<int32_t> levels;
  std::vector<ColItem> cols;
  std::vector<UpdItem> upds;
  std::vector<ChainItem> chains;
  std::vector<int32_t> chaincls;
  p->lvl_ptr.assign(H + 1, 0);
  p->col_ptr.assign(H + 1, 0);
  p->upd_ptr.assign(H + 1, 0);
  p->chain_ptr.assign(H + 1, 0);
  p->chaincl_ptr.assign(H + 1, 0);
  p->rhs_lds_fwd.assign(H + 1, 0);
  p->rhs_lds_back.assign(H + 1, 0);
  p->rhs_big.assign(H + 1, 0);
  p->groups.assign((H + 1) * ndg_plan::kClasses, ndg_plan::Group{});
  auto class_of = [&](int k) { return size_class(sy, k); };
  for (int h = 1; h <= H; ++h) {
    std::vector<int32_t> lv(sy.level_order.begin() + sy.level_ptr[h - 1],
                            sy.level_order.begin() + sy.level_ptr[h]);
    std::stable_sort(lv.begin(), lv.end(), [&](int32_t a, int32_t b) { return class_of(a) < class_of(b); });
    for (int q = 0; q < ndg_plan::kClasses; ++q) {
      ndg_plan::Group& g = p->groups[h * ndg_plan::kClasses + q];
      g.cl0 = (int)levels.size();
      g.col0 = (int)cols.size();
      g.upd0 = (int)upds.size();
      for (int32_t k : lv) {
        if (class_of(k) != q) continue;
        const int s_ = sy.s(k), b = sy.b(k);
        levels.push_back(k);
        g.ncl++;
        if (q <= 2) {
          g.size = std::max(g.size, s_ + b);
          // Psi and X_{i,B} rows padded to an odd stride (bank spread);
          // the upper triangle of X_{B,B}, later X_ii
          const size_t full = (size_t)(2 * s_ * (b | 1) + std::max(b * (b + 1) / 2, s_ * (s_ | 1))) * 16;
          g.lds = std::max(g.lds, full);
          // without phonon sources a leaf off the contact chains keeps X_{i,B}
          // in the space of X_{B,B} (the kernel's test, with this front's own
          // block size: a larger group front only raises the items' bound)
          const int nt = extract_threads(s_ + b);
          const bool leaf_layout = sy.children[k].empty() && p->hdesc[k].chain_mask == 0 &&
                                   ((s_ + 1) / 2) * b <= extract_leaf_items(nt) * nt;
          g.lds_leaf = std::max(g.lds_leaf, leaf_layout ? (size_t)(s_ * (b | 1) + std::max(b * (b + 1) / 2, s_ * (b | 1))) * 16 : full);
        } else {
          g.size = std::max(g.size, s_);
          const int nt = (b + 63) / 64;
          for (int tc = 0; tc < nt; ++tc) cols.push_back(ColItem{k, tc});
          // class 3 (s <= 16) updates in 32-row tiles; the contribution is
          // symmetric, so tiles wholly below its diagonal are skipped
          const int tmr = q == 3 ? 32 : 64;
          const int ntr = (b + tmr - 1) / tmr;
          for (int tr = 0; tr < ntr; ++tr)
            for (int tc = 0; tc < nt; ++tc)
              if (tr * tmr <= tc * 64 + 63) upds.push_back(UpdItem{k, tr, tc, 0});
        }
      }
      g.ncol = (int)cols.size() - g.col0;
      g.nupd = (int)upds.size() - g.upd0;
    }
    for (int32_t k : lv) {
      const int s_ = sy.s(k), b = sy.b(k);
      if (rhs_small_host(s_, b)) {
        p->rhs_lds_fwd[h] = std::max(p->rhs_lds_fwd[h], std::max<size_t>(16, rhs_small_lds_fwd(s_, b)));
        p->rhs_lds_back[h] = std::max(p->rhs_lds_back[h], rhs_small_lds_back(s_, b));
      } else {
        p->rhs_big[h] = 1;
      }
    }
    for (int32_t k : lv)
      if (p->hdesc[k].chain_mask) {
        chaincls.push_back(k);
        for (int c = 0; c < p->ncontacts; ++c)
          if ((p->hdesc[k].chain_mask >> c) & 1) chains.push_back(ChainItem{k, c});
      }
    p->lvl_ptr[h] = (int)levels.size();
    p->col_ptr[h] = (int)cols.size();
    p->upd_ptr[h] = (int)upds.size();
    p->chain_ptr[h] = (int)chains.size();
    p->chaincl_ptr[h] = (int)chaincls.size();
  }
  phonon_free_costs(sy, p->hdesc, p->nc, p->ncontacts, p->cost_flops, p->cost_bytes);
  std::vector<int32_t> kids_ptr(nc + 1, 0), kids;
  for (int k = 0; k < nc; ++k) {
    for (int32_t ch : sy.children[k]) kids.push_back(ch);
    kids_ptr[k + 1] = (int32_t)kids.size();
  }
  // front assembly: -H rows, self-energy maps, children's index maps
  std::vector<double> hfront;
  std::vector<int32_t> smap, pinv;
  for (int k = 0; k < nc; ++k) {
    ClusterDesc& d = p->hdesc[k];
    d.o_hf = d.o_smap = d.o_pinv = -1;
    const int s_ = d.s, f = d.f;
    {
      d.o_hf = (int64_t)hfront.size();
      hfront.resize(hfront.size() + (size_t)s_ * f, 0.0);
      double* hf = hfront.data() + d.o_hf;
      for (int64_t q = sy.hptr[k]; q < sy.hptr[k + 1]; ++q) hf[(int64_t)sy.hrow[q] * f + sy.hcol[q]] -= sy.hval[q];
      if (sy.sptr[k] < sy.sptr[k + 1]) {
        d.o_smap = (int64_t)smap.size();
        smap.resize(smap.size() + (size_t)f * f, -1);
        int32_t* sm = smap.data() + d.o_smap;
        for (int64_t q = sy.sptr[k]; q < sy.sptr[k + 1]; ++q)
          sm[(int64_t)sy.srow[q] * f + sy.scol[q]] = (sy.scid[q] << 24) | sy.sflat[q];
      }
    }
    const int par = sy.parent[k];
    if (par >= 0) {
      const int fp = sy.s(par) + sy.b(par);
      d.o_pinv = (int64_t)pinv.size();
      pinv.resize(pinv.size() + fp, -1);
      for (int r = 0; r < d.b; ++r) pinv[d.o_pinv + sy.relmap[sy.bptr[k] + r]] = r;
    }
  }
  // extraction gather tables (see ClusterDesc::o_gaddr): entry (u, v) of
  // X_{B,B} sits in the stored rows of the lower of the clusters owning B[u]
  // and B[v] (B[u], B[v] are coupled after fill, so the other point is in
  // that cluster's front)
  std::vector<int32_t> gaddr;
  const int64_t pdelta = p->hdesc.empty() ? 0 : p->hdesc[0].o_fp - p->hdesc[0].o_fg;
  if (2 * pdelta >= (int64_t)1 << 31) {
    set_error("ndg_plan_create: fronts exceed the 2^31-entry gather range");
    free_plan(p);
    return NDG_EINVAL;
  }
  // slab offset of G^r(x, y) for coupled points x, y: the stored rows of the
  // lower owning cluster, bit 31 set when stored as G^r(y, x); false if y is
  // missing from that cluster's front
  auto stored_addr = [&](int32_t x0, int32_t y0, int32_t& out) {
    const int ou = sy.owner[x0], ov = sy.owner[y0];
    const bool direct = ou <= ov;  // post-order: the lower cluster has the smaller id
    const int a = direct ? ou : ov;
    const int32_t x = direct ? x0 : y0, y = direct ? y0 : x0;
    int pos;
    if (sy.owner[y] == a) pos = y - sy.cl_off[a];
    else {
      const int32_t* Ba0 = sy.bidx.data() + sy.bptr[a];
      const int32_t* Ba1 = sy.bidx.data() + sy.bptr[a + 1];
      const int32_t* it = std::lower_bound(Ba0, Ba1, y);
      if (it == Ba1 || *it != y) return false;
      pos = sy.s(a) + (int)(it - Ba0);
    }
    const ClusterDesc& da = p->hdesc[a];
    const int64_t o = da.o_fg + (int64_t)(x - sy.cl_off[a]) * da.f + pos;
    out = (int32_t)o | (direct ? 0 : (int32_t)0x80000000);
    return true;
  };
  for (int k = 0; k < nc; ++k) {
    ClusterDesc& d = p->hdesc[k];
    d.o_gaddr = (int64_t)gaddr.size();
    d.o_bbd = -1;
    d.bbd_ld = 0;
    const int b = d.b;
    if (b == 0) continue;
    const int32_t* B = sy.bidx.data() + sy.bptr[k];
    {
      // B a run of consecutive points of one cluster a: X_{B,B} is the
      // block of a's stored rows at (t0, t0), t0 = B[0] - a's first point
      const int a = sy.owner[B[0]];
      bool run = sy.owner[B[b - 1]] == a;
      for (int u = 1; u < b && run; ++u) run = B[u] == B[0] + u;
      if (run) {
        const int64_t t0 = B[0] - sy.cl_off[a];
        d.o_bbd = p->hdesc[a].o_fg + t0 * p->hdesc[a].f + t0;
        d.bbd_ld = p->hdesc[a].f;
      }
    }
    gaddr.resize(gaddr.size() + (size_t)b * b);
    int32_t* ga = gaddr.data() + d.o_gaddr;
    for (int u = 0; u < b; ++u)
      for (int v = 0; v < b; ++v)
        if (!stored_addr(B[u], B[v], ga[(int64_t)u * b + v])) {
          set_error("internal: boundary entry missing from an ancestor's front");
          free_plan(p);
          return NDG_EINVAL;
        }
  }
  // the contact blocks (terminal currents): entry (a, b) of contact c at
  // caddr[off_c + a nc + b], contact sites in the caller's order (every pair
  // of sites of one contact is coupled through its dense self-energy)
  std::vector<int32_t> caddr;
  for (int cc = 0; cc < p->ncontacts; ++cc) {
    const std::vector<int32_t>& cp = sy.contact_pos[cc];
    const size_t m = cp.size(), o0 = caddr.size();
    caddr.resize(o0 + m * m);
    for (size_t a = 0; a < m; ++a)
      for (size_t b = 0; b < m; ++b)
        if (!stored_addr(cp[a], cp[b], caddr[o0 + a * m + b])) {
          set_error("internal: contact entry missing from its clusters' fronts");
          free_plan(p);
          return NDG_EINVAL;
        }
  }
  // the assembly relies on the parent's points leading each sorted B
  for (int k = 0; k < nc; ++k) {
    const ClusterDesc& d = p->hdesc[k];
    for (int64_t q = sy.bptr[k] + d.nself; q < sy.bptr[k + 1]; ++q)
      if (sy.owner[sy.bidx[q]] == d.parent) {
        set_error("internal: parent's points do not lead a boundary set");
        free_plan(p);
        return NDG_EINVAL;
      }
  }
  std::vector<SiteDiag> sdiag(sy.n);
  for (int64_t pn = 0; pn < sy.n; ++pn) {
    const int k = sy.owner[pn];
    const ClusterDesc& d = p->hdesc[k];
    const int64_t r = pn - sy.cl_off[k];
    sdiag[sy.perm[pn]] = SiteDiag{d.o_fg + r * d.f + r, d.o_fp + r * d.f + r, k, 0};
  }
  for (int k = 0; k < nc; ++k)
    if ((int)sy.children[k].size() > kMaxKids) {
      set_error("ndg_plan_create: a cluster has more than 64 children");
      free_plan(p);
      return NDG_EINVAL;
    }
  for (int k = 0; k < nc; ++k)
    for (int64_t q = sy.sptr[k]; q < sy.sptr[k + 1]; ++q)
      if (sy.sflat[q] >= (1 << 24)) {
        set_error("ndg_plan_create: contact too large for the self-energy index map");
        free_plan(p);
        return NDG_EINVAL;
      }
  int rc = 0;
  rc = rc ? rc : upload(&p->d_cl, p->hdesc.data(), p->hdesc.size());
  rc = rc ? rc : upload(&p->d_relmap, sy.relmap.data(), sy.relmap.size());
  rc = rc ? rc : upload(&p->d_kids_ptr, kids_ptr.data(), kids_ptr.size());
  rc = rc ? rc : upload(&p->d_kids, kids.data(), kids.size());
  rc = rc ? rc : upload(&p->d_hfront, hfront.data(), hfront.size());
  rc = rc ? rc : upload(&p->d_smap, smap.data(), smap.size());
  rc = rc ? rc : upload(&p->d_pinv, pinv.data(), pinv.size());
  rc = rc ? rc : upload(&p->d_gaddr, gaddr.data(), gaddr.size());
  rc = rc ? rc : upload(&p->d_caddr, caddr.data(), caddr.size());
  // sources of the separate G^> step and of the transmission, per batch
  for (int c = 0; c < p->ncontacts && !rc; ++c)
    if (hipMalloc((void**)&p->d_src[c], (size_t)max_batch * p->nc[c] * p->nc[c] * 16) != hipSuccess) rc = NDG_ENOMEM;
  rc = rc ? rc : upload(&p->d_sdiag, sdiag.data(), sdiag.size());
  rc = rc ? rc : upload(&p->d_hrow, sy.hrow.data(), sy.hrow.size());
  rc = rc ? rc : upload(&p->d_hcol, sy.hcol.data(), sy.hcol.size());
  rc = rc ? rc : upload(&p->d_hval, sy.hval.data(), sy.hval.size());
  rc = rc ? rc : upload(&p->d_perm, sy.perm.data(), sy.perm.size());
  rc = rc ? rc : upload(&p->d_owner, sy.owner.data(), sy.owner.size());
  {
    std::vector<int32_t> cinv(p->n, -1);
    int32_t col = 0;
    for (int c = 0; c < p->ncontacts && !rc; ++c) {
      rc = upload(&p->d_cpos[c], sy.contact_pos[c].data(), sy.contact_pos[c].size());
      for (size_t a = 0; a < sy.contact_pos[c].size(); ++a) cinv[sy.contact_pos[c][a]] = col++;
    }
    rc = rc ? rc : upload(&p->d_cinv, cinv.data(), cinv.size());
  }
  rc = rc ? rc : upload(&p->d_srow, sy.srow.data(), sy.srow.size());
  rc = rc ? rc : upload(&p->d_scol, sy.scol.data(), sy.scol.size());
  rc = rc ? rc : upload(&p->d_scid, sy.scid.data(), sy.scid.size());
  rc = rc ? rc : upload(&p->d_sflat, sy.sflat.data(), sy.sflat.size());
  rc = rc ? rc : upload(&p->d_levels, levels.data(), levels.size());
  rc = rc ? rc : upload(&p->d_colitems, cols.data(), cols.size());
  rc = rc ? rc : upload(&p->d_upditems, upds.data(), upds.size());
  rc = rc ? rc : upload(&p->d_chainitems, chains.data(), chains.size());
  rc = rc ? rc : upload(&p->d_chaincls, chaincls.data(), chaincls.size());
  if (!rc) {
    const size_t bytes = (size_t)p->stride * 16 * (size_t)max_batch;
    if (hipMalloc((void**)&p->d_ws, bytes) != hipSuccess) rc = NDG_ENOMEM;
  }
  if (!rc) {
    if (hipMalloc((void**)&p->d_status, 4 * sizeof(int32_t)) != hipSuccess) rc = NDG_ENOMEM;
    else if (hipMemset(p->d_status, 0, 4 * sizeof(int32_t)) != hipSuccess) rc = NDG_EHIP;
  }
  if (!rc) {
    // default priority, like every stream of the library
    if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&p->chain, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess)
      rc = NDG_EHIP;
    p->ev_chain.assign(p->max_height + 1, nullptr);
    for (int h = 1; h <= p->max_height && !rc; ++h)
      if (p->chaincl_ptr[h] > p->chaincl_ptr[h - 1] &&
          hipEventCreateWithFlags(&p->ev_chain[h], hipEventDisableTiming) != hipSuccess)
        rc = NDG_EHIP;
  }
  if (rc) {
    (void)hipGetLastError();
    free_plan(p);
    set_error(rc == NDG_ENOMEM ? "ndg_plan_create: device allocation failed" : "ndg_plan_create: HIP copy failed");
    return rc;
  }
  std::memset(&p->info, 0, sizeof(p->info));
  p->info.n = sy.n;
  p->info.nclusters = nc;
  p->info.max_height = H;
  p->info.max_cluster = sy.max_cluster;
  p->info.max_boundary = sy.max_boundary;
  p->info.ncontacts = p->ncontacts;
  p->info.nnz_boundary = (int64_t)sy.bidx.size();
  p->info.ops_fold_inv = oc.fold_inv;
  p->info.ops_fold_psi = oc.fold_psi;
  p->info.ops_fold_update = oc.fold_update;
  p->info.ops_gr_off = oc.gr_off;
  p->info.ops_gr_diag = oc.gr_diag;
  p->info.ops_gl_chain = oc.gl_chain;
  p->info.ops_gl_off = oc.gl_off;
  p->info.ops_gl_diag = oc.gl_diag;
  p->info.ops_total = oc.total();
  p->info.workspace_bytes_per_energy = p->stride * 16;
  *out = p;
  return NDG_OK;
}

int plan_destroy(ndg_plan* plan) {
  if (!plan) return NDG_OK;
  // solves still in flight (on the caller's stream or the plan's own) use
  // the workspace and tables freed below
  if (hipSetDevice(plan->device) == hipSuccess) (void)hipDeviceSynchronize();
  free_plan(plan);
  return NDG_OK;
}

int plan_info(const ndg_plan* plan, ndg_info* out) {
  *out = plan->info;
  return NDG_OK;
}

int plan_enable_adjoint(ndg_plan* p) {
  if (p->d_rX) return NDG_OK;
  for (int k = 0; k < p->nclusters; ++k)
    if (p->hdesc[k].s > kMaxClusterAux) {
      set_error("ndg_plan_enable_adjoint: the adjoint's solves take clusters of at most 64 points");
      return NDG_EINVAL;
    }
  if (hipSetDevice(p->device) != hipSuccess) { set_error("ndg_plan_enable_adjoint: hipSetDevice failed"); return NDG_EHIP; }
  // one right-hand side with the columns of all contacts side by side
  int mmax = 0;
  for (int c = 0; c < p->ncontacts; ++c) mmax += p->nc[c];
  mmax = std::max(mmax, 1);
  std::vector<int64_t> ovec(p->nclusters);
  int64_t off = 0;
  for (int k = 0; k < p->nclusters; ++k) {
    ovec[k] = off;
    off += align8((int64_t)p->hdesc[k].f * mmax);
  }
  p->zstride = off;
  p->mmax = mmax;
  const size_t nb = (size_t)p->max_batch, nm = (size_t)p->n * mmax;
  int rc = 0;
  if (hipMalloc((void**)&p->d_rX, nb * nm * 16) != hipSuccess ||
      hipMalloc((void**)&p->d_rG, nb * nm * 16) != hipSuccess ||
      hipMalloc((void**)&p->d_rZ, nb * (size_t)p->zstride * 16) != hipSuccess ||
      hipMalloc((void**)&p->d_part, nb * (size_t)p->n * 8) != hipSuccess ||
      hipMalloc((void**)&p->d_pvec, (size_t)ndg_plan::kPoissonVecs * (size_t)p->n * 8) != hipSuccess ||
      hipMalloc((void**)&p->d_pdot, (size_t)(kVecBlocks + 2) * 8) != hipSuccess)
    rc = NDG_ENOMEM;
  if (!rc) rc = upload(&p->d_ovec, ovec.data(), ovec.size());
  if (!rc) rc = upload(&p->d_bidx, p->hbidx.data(), p->hbidx.size());
  if (rc) {
    (void)hipGetLastError();
    void* ptrs[] = {p->d_rX, p->d_rG, p->d_rZ, p->d_part, p->d_ovec, p->d_bidx, p->d_pvec, p->d_pdot};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    p->d_rX = p->d_rG = p->d_rZ = nullptr;
    p->d_part = nullptr;
    p->d_pvec = p->d_pdot = nullptr;
    p->d_ovec = nullptr;
    p->d_bidx = nullptr;
    set_error("ndg_plan_enable_adjoint: device allocation failed");
    return rc;
  }
  return NDG_OK;
}

int plan_enable_scattering(ndg_plan* p) {
  static_assert(kClusterRows >= kMaxClusterAux, "scattering kernels stage one value per cluster row");
  if (p->d_sws) return NDG_OK;
  for (int k = 0; k < p->nclusters; ++k)
    if (p->hdesc[k].s > kMaxClusterAux) {
      set_error("ndg_plan_enable_scattering: the scattering kernels take clusters of at most 64 points");
      return NDG_EINVAL;
    }
  if (hipSetDevice(p->device) != hipSuccess) {
    set_error("ndg_plan_enable_scattering: hipSetDevice failed");
    return NDG_EHIP;
  }
  const int nc = p->nclusters, H = p->max_height;
  const auto& hd = p->hdesc;
  // frames: the cluster, then its ancestors parent first
  std::vector<ScatDesc> sd(nc);
  std::vector<int32_t> atab;
  std::vector<std::vector<int32_t>> chain(nc), ao(nc);
  int64_t off = 0;
  for (int i = 0; i < nc; ++i) {
    for (int k = i; k >= 0; k = hd[k].parent) chain[i].push_back(k);
    const int D = (int)chain[i].size() - 1;
    if (D > kMaxAncestors) {
      set_error("ndg_plan_enable_scattering: tree deeper than 63 ancestors");
      return NDG_EINVAL;
    }
    ao[i].assign(D + 2, 0);
    for (int t = 0; t <= D; ++t) ao[i][t + 1] = ao[i][t] + hd[chain[i][t]].s;
    sd[i] = ScatDesc{off, ao[i][D + 1], D, (int32_t)atab.size(), 0, 0, 0};
    atab.insert(atab.end(), chain[i].begin(), chain[i].end());
    atab.insert(atab.end(), ao[i].begin(), ao[i].end());
    off += align8((int64_t)hd[i].s * sd[i].g);
  }
  std::vector<int32_t> owner(p->n);
  for (int i = 0; i < nc; ++i)
    for (int r = 0; r < hd[i].s; ++r) owner[hd[i].pt_off + r] = i;
  // B entries in the frame; descendants feeding each cluster's N rows
  std::vector<BPos> bpos(p->hbidx.size());
  std::vector<std::vector<LkItem>> lkj(nc);
  std::vector<int32_t> umap;
  for (int i = 0; i < nc; ++i) {
    const int b = hd[i].b;
    for (int u = 0; u < b; ++u) {
      const int xpt = p->hbidx[hd[i].bptr + u], o = owner[xpt];
      int t = 1;
      while (t < (int)chain[i].size() && chain[i][t] != o) ++t;
      if (t >= (int)chain[i].size()) {
        set_error("ndg_plan_enable_scattering: boundary point outside the ancestors");
        return NDG_EINVAL;
      }
      bpos[hd[i].bptr + u] = BPos{ao[i][t] + xpt - hd[o].pt_off, t};
    }
    // B is ascending and every cluster's points are contiguous: one run per owner
    for (int u0 = 0; u0 < b;) {
      const int a = bpos[hd[i].bptr + u0].a, j = chain[i][a];
      int u1 = u0;
      const int moff = (int)umap.size();
      umap.resize(moff + hd[j].s, -1);
      while (u1 < b && bpos[hd[i].bptr + u1].a == a) {
        umap[moff + p->hbidx[hd[i].bptr + u1] - hd[j].pt_off] = u1;
        ++u1;
      }
      lkj[j].push_back(LkItem{i, moff, ao[i][a], 0});
      u0 = u1;
    }
  }
  std::vector<LkItem> lk;
  for (int j = 0; j < nc; ++j) {
    sd[j].lk0 = (int32_t)lk.size();
    lk.insert(lk.end(), lkj[j].begin(), lkj[j].end());
    sd[j].lk1 = (int32_t)lk.size();
  }
  // launch lists per height and tile class; the algorithmic work per energy
  std::vector<ColItem> items;
  std::vector<int32_t> cls;
  p->anc_groups.assign((H + 1) * 3, ndg_plan::AncGroup{});
  for (int h = 1; h <= H; ++h)
    for (int q = 0; q < 3; ++q) {
      ndg_plan::AncGroup& g = p->anc_groups[h * 3 + q];
      g.it0 = (int)items.size();
      g.cl0 = (int)cls.size();
      for (int i = 0; i < nc; ++i) {
        const int si = hd[i].s, qi = si <= 16 ? 0 : si <= 32 ? 1 : 2;
        if (p->hheight[i] != h || qi != q) continue;
        cls.push_back(i);
        for (int tc = 0; tc * 64 < sd[i].g; ++tc) items.push_back(ColItem{i, tc});
      }
      g.nit = (int)items.size() - g.it0;
      g.ncl = (int)cls.size() - g.cl0;
    }
  for (int i = 0; i < nc; ++i) {
    const int h = p->hheight[i];
    const double s = hd[i].s, b = hd[i].b, f = hd[i].f, g = sd[i].g, W = g - s;
    const int q = hd[i].s <= 16 ? 0 : hd[i].s <= 32 ? 1 : 2;  // the launch's tile class
    p->cost_flops[cost_index(K_ANC_G, h, q, H)] += 8.0 * s * b * W;
    p->cost_bytes[cost_index(K_ANC_G, h, q, H)] += 16.0 * (s * b + b * W + s * g);
    // the N fold of an inner cluster: read G^(0) rows, write N, and per
    // feeding descendant its N rows over this frame and its Psi entries
    // (leaves are formed inside k_anc_g: no launch, no cost here)
    if (h > 1) {
      double nf = 0, nby = 32.0 * s * g;
      for (const LkItem& L : lkj[i]) {
        nf += 8.0 * s * hd[L.d].s * g;
        nby += 16.0 * hd[L.d].s * (g + s);
      }
      p->cost_flops[cost_index(K_ANC_N, h, q, H)] += nf;
      p->cost_bytes[cost_index(K_ANC_N, h, q, H)] += nby;
    }
    p->cost_flops[cost_index(K_ANC_P0, h, q, H)] += 8.0 * s * s * f;
    p->cost_bytes[cost_index(K_ANC_P0, h, q, H)] += 16.0 * (s * s + 2.0 * s * f);
  }
  p->sstride = off;
  int rc = 0;
  if (hipMalloc((void**)&p->d_sws, (size_t)p->max_batch * (size_t)off * 16) != hipSuccess) rc = NDG_ENOMEM;
  if (!rc) rc = upload(&p->d_sd, sd.data(), sd.size());
  if (!rc) rc = upload(&p->d_atab, atab.data(), atab.size());
  if (!rc && !bpos.empty()) rc = upload(&p->d_bpos, bpos.data(), bpos.size());
  if (!rc && !lk.empty()) rc = upload(&p->d_lk, lk.data(), lk.size());
  if (!rc && !umap.empty()) rc = upload(&p->d_umap, umap.data(), umap.size());
  if (!rc) rc = upload(&p->d_ancitems, items.data(), items.size());
  if (!rc) rc = upload(&p->d_anccls, cls.data(), cls.size());
  if (!rc && hipMalloc((void**)&p->d_scba, (2 * kScbaBlocks + 2) * sizeof(double)) != hipSuccess) rc = NDG_ENOMEM;
  if (rc) {
    (void)hipGetLastError();
    void* ptrs[] = {p->d_sws, p->d_sd, p->d_atab, p->d_bpos, p->d_lk, p->d_umap, p->d_ancitems, p->d_anccls,
                    p->d_scba};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    p->d_sws = nullptr;
    p->d_sd = nullptr;
    p->d_atab = nullptr;
    p->d_bpos = nullptr;
    p->d_lk = nullptr;
    p->d_umap = nullptr;
    p->d_ancitems = nullptr;
    p->d_anccls = nullptr;
    p->d_scba = nullptr;
    for (int k = K_ANC_G; k <= K_ANC_P0; ++k)
      for (int h = 0; h <= H; ++h)
        for (int q = 0; q < kCostClasses; ++q)
          p->cost_flops[cost_index(k, h, q, H)] = p->cost_bytes[cost_index(k, h, q, H)] = 0;
    set_error("ndg_plan_enable_scattering: device allocation failed");
    return rc == NDG_ENOMEM ? NDG_ENOMEM : rc;
  }
  p->info.scatter_bytes_per_energy = off * 16;
  return NDG_OK;
}

int plan_solve(ndg_plan* p, int nE, const double* E, double eta, const double* V,
               const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, ndg_c128* dgr,
               ndg_c128* dgl, ndg_c128* dgg, double* growth, int prec, void* stream) {
  return plan_run(p, kRunSolve, nE, E, eta, V, sig_r, sig_less, dgr, dgl, dgg, growth, nullptr,
                  nullptr, nullptr, nullptr, prec, stream);
}

int plan_scba(ndg_plan* p, int nE, const double* E, double eta, const double* V,
              const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, double d0, double mix,
              double tol, int max_iter, ndg_c128* sig_r_ph, ndg_c128* sig_less_ph, ndg_c128* dgr,
              ndg_c128* dgl, ndg_c128* dgg, double* current, int32_t* iterations, double* residual,
              void* stream) {
  if (!p->d_sws) {
    set_error("ndg_scba: call ndg_plan_enable_scattering first");
    return NDG_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  int it = 0;
  double res = 0.0, hm[2] = {0.0, 0.0};
  while (it < max_iter) {
    int rc = plan_run(p, kRunSolve, nE, E, eta, V, sig_r, sig_less, dgr, dgl, dgg, nullptr, nullptr, nullptr,
                      nullptr, nullptr, NDG_FP64, stream, nullptr, sig_r_ph, sig_less_ph, current);
    if (rc) return rc;
    ++it;
    launch_scba_mix(reinterpret_cast<const double2*>(dgr), reinterpret_cast<const double2*>(dgl),
                    reinterpret_cast<double2*>(sig_r_ph), reinterpret_cast<double2*>(sig_less_ph),
                    (int64_t)nE * p->n, d0, mix, p->d_scba, p->d_scba + 2 * kScbaBlocks, st);
    if (hipMemcpyAsync(hm, p->d_scba + 2 * kScbaBlocks, sizeof(hm), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("ndg_scba: reading the residual failed");
      return NDG_EHIP;
    }
    res = hm[1] > 0.0 ? hm[0] / hm[1] : 0.0;
    if (res < tol) break;
  }
  if (iterations) *iterations = it;
  if (residual) *residual = res;
  return NDG_OK;
}

int plan_poisson_newton(ndg_plan* p, int nE, const double* E, double eta, const double* V,
                        const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, const double* cE,
                        const int64_t* k_rowptr, const int32_t* k_col, const double* k_val, int64_t k_nnz,
                        double beta, const double* nd, double cg_tol, int cg_max_iter, double* delta,
                        double* res_norm, int32_t* cg_iterations, double* cg_residual, void* stream) {
  if (!p->d_pvec) {
    set_error("ndg_poisson_newton_step: call ndg_plan_enable_adjoint first");
    return NDG_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = p->n;
  double* nv = p->d_pvec;       // n(V), then K p
  double* F = nv + n;           // residual
  double* r = F + n;
  double* pv = r + n;
  double* chip = pv + n;        // chi p (the density's vector-Jacobian product with p)
  double* Ap = chip + n;
  double* kv = Ap + n;
  double* part = p->d_pdot;
  double* dot = part + kVecBlocks;
  auto dot_host = [&](const double* a, const double* b, double& out) {
    launch_dot(n, a, b, part, dot, st);
    if (hipMemcpyAsync(&out, dot, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      set_error("ndg_poisson_newton_step: reading a dot product failed");
      return false;
    }
    return true;
  };
  // F = K V - beta (n(V) - n_D)
  int rc = plan_run(p, kRunDensity, nE, E, eta, V, sig_r, sig_less, nullptr, nullptr, nullptr, nullptr, cE, nv,
                    nullptr, nullptr, NDG_FP64, stream);
  if (rc) return rc;
  launch_spmv(n, k_nnz, k_rowptr, k_col, k_val, V, kv, st);
  launch_axpby(n, 1.0, nv, -1.0, nd, nv, st);
  launch_axpby(n, 1.0, kv, -beta, nv, F, st);
  // conjugate gradients on J delta = -F, J = K - beta chi (chi symmetric in
  // equilibrium, so chi p is the vector-Jacobian product with p)
  launch_axpby(n, -1.0, F, 0.0, F, r, st);
  launch_axpby(n, 1.0, r, 0.0, r, pv, st);
  launch_axpby(n, 0.0, r, 0.0, r, delta, st);
  double rr = 0.0;
  if (!dot_host(r, r, rr)) return NDG_EHIP;
  const double f0 = std::sqrt(rr);
  if (res_norm) *res_norm = f0;
  int it = 0;
  double rel = f0 > 0.0 ? 1.0 : 0.0;
  // V and the energies stay fixed during the step: when they fit one batch,
  // the density solve's factors serve every vector-Jacobian product (its
  // extraction writes only the fronts' rows, the solves read only Psi and the
  // pivot inverses)
  const bool reuse = nE <= p->max_batch;
  while (it < cg_max_iter && rel > cg_tol) {
    rc = plan_run(p, kRunVjp, nE, E, eta, V, sig_r, sig_less, nullptr, nullptr, nullptr, nullptr, cE, nullptr,
                  pv, chip, NDG_FP64, stream, nullptr, nullptr, nullptr, nullptr, reuse);
    if (rc) return rc;
    launch_spmv(n, k_nnz, k_rowptr, k_col, k_val, pv, kv, st);
    launch_axpby(n, 1.0, kv, -beta, chip, Ap, st);
    double pap = 0.0;
    if (!dot_host(pv, Ap, pap)) return NDG_EHIP;
    if (!(pap > 0.0)) {
      set_error("ndg_poisson_newton_step: the Jacobian is not positive definite along a search direction");
      return NDG_ENOTSPD;
    }
    const double alpha = rr / pap;
    launch_axpby(n, 1.0, delta, alpha, pv, delta, st);
    launch_axpby(n, 1.0, r, -alpha, Ap, r, st);
    double rr_new = 0.0;
    if (!dot_host(r, r, rr_new)) return NDG_EHIP;
    ++it;
    rel = std::sqrt(rr_new) / f0;
    launch_axpby(n, 1.0, r, rr_new / rr, pv, pv, st);
    rr = rr_new;
  }
  if (cg_iterations) *cg_iterations = it;
  if (cg_residual) *cg_residual = rel;
  if (hipGetLastError() != hipSuccess) {
    set_error("ndg_poisson_newton_step: kernel launch failed");
    return NDG_EHIP;
  }
  return NDG_OK;
}

int plan_solve_chunk(ndg_plan* p, int nE, const double* E, double eta, const double* V,
                     const ndg_c128* const* sig_r, const ndg_c128* const* sig_less,
                     ndg_c128* dgr, ndg_c128* dgl, ndg_c128* dgg, double* growth, int prec,
                     void* stream, const int32_t* e0p) {
  return plan_run(p, kRunSolve, nE, E, eta, V, sig_r, sig_less, dgr, dgl, dgg, growth, nullptr,
                  nullptr, nullptr, nullptr, prec, stream, e0p);
}

int plan_max_batch(const ndg_plan* p) { return p->max_batch; }

int plan_run(ndg_plan* p, int mode, int nE, const double* E, double eta, const double* V,
             const ndg_c128* const* sig_r, const ndg_c128* const* sig_less, ndg_c128* dgr,
             ndg_c128* dgl, ndg_c128* dgg, double* growth, const double* cE, double* density,
             const double* nbar, double* vbar, int prec, void* stream, const int32_t* e0p,
             const ndg_c128* sig_r_ph, const ndg_c128* sig_less_ph, double* current, bool reuse_fold,
             double* vjp_part, int64_t vjp_part_capacity, ndg_c128* dgg_explicit, double* transmission) {
  const bool scat = sig_less_ph != nullptr;
  if ((dgg_explicit || transmission) && (mode != kRunSolve || scat || e0p)) {
    set_error("internal: the separate G^> step and the transmission are for plain solves only");
    return NDG_EINVAL;
  }
  if (transmission && p->ncontacts != 2) {
    set_error("ndg_solve_transport: the transmission needs two contacts");
    return NDG_EINVAL;
  }
  if ((scat || sig_r_ph) && (mode != kRunSolve || e0p || prec != NDG_FP64)) {
    set_error("internal: phonon self-energies are for FP64 solves only");
    return NDG_EINVAL;
  }
  if (scat && !p->d_sws) {
    set_error("ndg_solve_scattering: call ndg_plan_enable_scattering first");
    return NDG_EINVAL;
  }
  if (e0p && mode != kRunSolve) {
    set_error("internal: device-resident energy offsets are for solves only");
    return NDG_EINVAL;
  }
  if (prec != NDG_FP64 && prec != NDG_MIXED) {
    set_error("ndg_solve: unknown precision");
    return NDG_EINVAL;
  }
  if (p->ncontacts > 0 && (!sig_r || !sig_less)) {
    set_error("ndg_solve: contact self-energies missing");
    return NDG_EINVAL;
  }
  for (int c = 0; c < p->ncontacts; ++c)
    if (!sig_r[c] || !sig_less[c]) {
      set_error("ndg_solve: NULL contact self-energy pointer");
      return NDG_EINVAL;
    }
  if (hipSetDevice(p->device) != hipSuccess) { set_error("ndg_solve: hipSetDevice failed"); return NDG_EHIP; }
  hipStream_t st = (hipStream_t)stream;
  Ctx c{};
  c.cl = p->d_cl;
  c.relmap = p->d_relmap;
  c.kids_ptr = p->d_kids_ptr;
  c.kids = p->d_kids;
  c.hrow = p->d_hrow;
  c.hcol = p->d_hcol;
  c.hval = p->d_hval;
  c.srow = p->d_srow;
  c.scol = p->d_scol;
  c.scid = p->d_scid;
  c.sflat = p->d_sflat;
  c.hfront = p->d_hfront;
  c.smap = p->d_smap;
  c.pinv = p->d_pinv;
  c.gaddr = p->d_gaddr;
  c.pdelta = p->hdesc.empty() ? 0 : p->hdesc[0].o_fp - p->hdesc[0].o_fg;
  c.sdiag = p->d_sdiag;
  c.perm = p->d_perm;
  c.owner = p->d_owner;
  c.ncontacts = p->ncontacts;
  for (int q = 0; q < 2; ++q) {
    c.cpos[q] = p->d_cpos[q];
    c.nc[q] = p->nc[q];
    c.sig_r[q] = q < p->ncontacts ? reinterpret_cast<const double2*>(sig_r[q]) : nullptr;
    c.sig_l[q] = q < p->ncontacts ? reinterpret_cast<const double2*>(sig_less[q]) : nullptr;
  }
  c.n = (int32_t)p->n;
  c.ws = p->d_ws;
  c.stride = p->stride;
  c.E = E;
  c.e0p = e0p;
  c.nE = nE;
  c.eta = eta;
  c.V = V;
  c.status = p->d_status;
  c.growth = growth;
  c.mixed = prec == NDG_MIXED ? 1 : 0;
  c.sig_r_ph = reinterpret_cast<const double2*>(sig_r_ph);
  c.sig_l_ph = reinterpret_cast<const double2*>(sig_less_ph);
  c.scat = scat ? 1 : 0;
  ScatCtx x{p->d_sd, p->d_atab, p->d_bpos, p->d_lk, p->d_umap, p->d_sws, p->sstride};
  // a kernel, so graph capture stays valid; a chunk leaves it to the caller
  if (growth && !e0p) launch_fill_zero(growth, nE, st);
  if (mode == kRunDensity) launch_zero(density, p->n, st);
  if (mode == kRunVjp) {
    if (!p->d_rX) {
      set_error("ndg_density_vjp: call ndg_plan_enable_adjoint first");
      return NDG_EINVAL;
    }
    // the per-energy partials of one batch: the plan's buffer, or the
    // caller-supplied (static) one, which must hold them
    if (vjp_part && (int64_t)std::min(nE, p->max_batch) * p->n > vjp_part_capacity) {
      set_error("ndg_density_vjp_noalloc: n x min(nE, max_batch) = " +
                std::to_string((int64_t)std::min(nE, p->max_batch) * p->n) +
                " partials exceed the static buffer of " + std::to_string(vjp_part_capacity) + " doubles");
      return NDG_EINVAL;
    }
    launch_zero(vbar, p->n, st);
  }
  RhsCtx r{};
  r.X = p->d_rX;
  r.Gc = p->d_rG;
  r.Z = p->d_rZ;
  r.o_vec = p->d_ovec;
  r.zstride = p->zstride;
  r.n = (int32_t)p->n;
  r.bidx = p->d_bidx;
  r.nbar = nbar;
  r.part = vjp_part ? vjp_part : p->d_part;
  const int H = p->max_height;
  // profiling: an event pair around each launch, with its algorithmic work
  auto take_event = [&]() {
    hipEvent_t ev = nullptr;
    if (!p->event_pool.empty()) { ev = p->event_pool.back(); p->event_pool.pop_back(); }
    else (void)hipEventCreate(&ev);
    return ev;
  };
  // each launch is credited with its own group's work (kernel, height, class)
  auto timed_on = [&](hipStream_t on, int kid, int h, int q, int nb, auto&& launch) {
    if (!p->profiling) { launch(); return; }
    ndg_plan::Rec r{kid, h, q, take_event(), take_event(), p->cost_flops[cost_index(kid, h, q, H)] * nb,
                    p->cost_bytes[cost_index(kid, h, q, H)] * nb};
    (void)hipEventRecord(r.a, on);
    launch();
    (void)hipEventRecord(r.b, on);
    p->recs.push_back(r);
  };
  auto timed = [&](int kid, int h, int q, int nb, auto&& launch) { timed_on(st, kid, h, q, nb, launch); };
  // with e0p: exactly one batch, its first energy read on the device
  const int e_end = e0p ? std::min(nE, 1) : nE;
  for (int e0 = 0; e0 < e_end; e0 += p->max_batch) {
    const int nb = std::min(p->max_batch, e0p ? nE : nE - e0);
    c.e0 = e0;
    // reuse_fold: the factors (Psi, pivot inverses) of this single batch are
    // still in the workspace from a previous call with the same energies and V
    for (int h = 1; h <= H && !reuse_fold; ++h) {
      const ChainItem* chi = p->d_chainitems + p->chain_ptr[h - 1];
      const int nch = p->chain_ptr[h] - p->chain_ptr[h - 1];
      for (int q = 0; q < ndg_plan::kClasses; ++q) {
        const ndg_plan::Group& g = p->groups[h * ndg_plan::kClasses + q];
        if (!g.ncl) continue;
        const int32_t* cl = p->d_levels + g.cl0;
        if (q <= 2) {
          timed(K_FOLD_SMALL, h, q, nb, [&] { launch_fold_small(c, cl, g.ncl, nb, g.size, st); });
          continue;
        }
        timed(K_ASSEMBLE, h, q, nb, [&] { launch_assemble(c, cl, g.ncl, nb, st); });
        timed(K_FACTOR, h, q, nb, [&] { launch_factor(c, cl, g.ncl, nb, g.size, st); });
        if (g.ncol) timed(K_PSI, h, q, nb, [&] { launch_psi(c, p->d_colitems + g.col0, g.ncol, nb, g.size, st); });
        if (g.nupd)
          timed(K_UPDATE, h, q, nb, [&] { launch_update(c, p->d_upditems + g.upd0, g.nupd, nb, q == 3 ? 32 : 64, st); });
      }
      // the G^< source; the gradient's solves need only the factors
      if (nch && mode != kRunVjp) timed(K_CHAIN_FWD, h, 0, nb, [&] { launch_chain_fwd(c, chi, nch, nb, st); });
    }
    if (mode == kRunVjp) {
      launch_zero(r.part, (int64_t)nb * p->n, st);
      r.m = 0;
      for (int cc = 0; cc < p->ncontacts; ++cc) r.m += p->nc[cc];
      if (r.m > 0) {
        // two solves with the factors, all contacts' columns at once:
        // G_{:,c} = A^{-1} E_c, then X_c = A^{-1} (Lambda conj(G_{:,c}))
        for (int pass = 0; pass < 2; ++pass) {
          RhsCtx rr = r;
          rr.ymode = pass;
          rr.cinv = p->d_cinv;
          rr.X = pass == 0 ? r.Gc : r.X;
          for (int h = 1; h <= H; ++h)
            timed(K_RHS_FWD, h, 0, nb, [&] {
              launch_rhs_fwd(c, rr, p->d_levels + p->lvl_ptr[h - 1], p->lvl_ptr[h] - p->lvl_ptr[h - 1], nb,
                             p->rhs_lds_fwd[h], p->rhs_big[h], st);
            });
          for (int h = H; h >= 1; --h)
            timed(K_RHS_BACK, h, 0, nb, [&] {
              launch_rhs_back(c, rr, p->d_levels + p->lvl_ptr[h - 1], p->lvl_ptr[h] - p->lvl_ptr[h - 1], nb,
                              p->rhs_lds_back[h], p->rhs_big[h], st);
            });
        }
        for (int cc = 0, off = 0; cc < p->ncontacts; off += p->nc[cc], ++cc)
          timed(K_VJP, 0, 0, nb, [&] { launch_vjp_accum(c, r, cc, off, nb, st); });
      }
      launch_vjp_reduce(c, r, nb, cE, vbar, st);
      p->last_batch = nb;
      continue;
    }
    // extraction of one height, G^r (lesser = false) or G^< (true)
    auto extract = [&](int h, bool lesser, hipStream_t on) {
      for (int q = 0; q < ndg_plan::kClasses; ++q) {
        const ndg_plan::Group& g = p->groups[h * ndg_plan::kClasses + q];
        if (!g.ncl) continue;
        const int32_t* cl = p->d_levels + g.cl0;
        if (q <= 2) {
          timed_on(on, lesser ? K_EXTRACT_SMALL_P : K_EXTRACT_SMALL, h, q, nb,
                   [&] { launch_extract_small(c, cl, g.ncl, nb, g.lds, g.lds_leaf, g.size, lesser, on); });
          continue;
        }
        const ColItem* ci = p->d_colitems + g.col0;
        if (g.ncol)
          timed_on(on, lesser ? K_DOWN_OFF_P : K_DOWN_OFF_G, h, q, nb,
                   [&] { launch_down_off(c, ci, g.ncol, nb, lesser, g.size, on); });
        timed_on(on, lesser ? K_DOWN_DIAG_P : K_DOWN_DIAG_G, h, q, nb,
                 [&] { launch_down_diag(c, cl, g.ncl, nb, lesser, g.size, on); });
      }
    };
    if (scat) {
      // phonon sources on every cluster, all on the caller's stream: G^r
      // extraction, the contact chains' part of the source, the rows of
      // G^(0) over all ancestors (top-down), the N fold and P_init
      // (bottom-up), then the G^< extraction
      for (int h = H; h >= 1; --h) extract(h, false, st);
      timed(K_CHAIN_T, 0, 0, nb, [&] { launch_chain_t(c, p->d_chainitems, p->chain_ptr[H], nb, st); });
      for (int h = H; h >= 1; --h) {
        const int k0 = p->chaincl_ptr[h - 1], nck = p->chaincl_ptr[h] - k0;
        if (nck) timed(K_CHAIN_BACK, h, 0, nb, [&] { launch_chain_back(c, p->d_chaincls + k0, nck, nb, st); });
      }
      static const int kTile[3] = {16, 32, 64};
      for (int h = H; h >= 1; --h)
        for (int q = 0; q < 3; ++q) {
          const ndg_plan::AncGroup& g = p->anc_groups[h * 3 + q];
          if (g.nit)
            timed(K_ANC_G, h, q, nb,
                  [&] { launch_anc_g(c, x, p->d_ancitems + g.it0, g.nit, nb, kTile[q], h == 1, st); });
        }
      // leaves (height 1) stored their N in k_anc_g
      for (int h = 1; h <= H; ++h)
        for (int q = 0; q < 3; ++q) {
          const ndg_plan::AncGroup& g = p->anc_groups[h * 3 + q];
          if (g.nit && h > 1)
            timed(K_ANC_N, h, q, nb, [&] { launch_anc_n(c, x, p->d_ancitems + g.it0, g.nit, nb, kTile[q], st); });
          if (g.ncl)
            timed(K_ANC_P0, h, q, nb, [&] { launch_anc_p0(c, x, p->d_anccls + g.cl0, g.ncl, nb, kTile[q], st); });
        }
      for (int h = H; h >= 1; --h) extract(h, true, st);
      timed(K_EPILOGUE, 0, 0, nb, [&] {
        launch_epilogue(c, nb, reinterpret_cast<double2*>(dgr), reinterpret_cast<double2*>(dgl),
                        reinterpret_cast<double2*>(dgg), st);
      });
      if (current) launch_current(c, p->d_caddr, nb, current, st);
      p->last_batch = nb;
      continue;
    }
    // G^r extraction on st, G^< extraction on the side stream (they write
    // disjoint buffers and read the fold's factors only), joined before the
    // epilogue.  The chain back substitution reads only the fold's factors
    // and its parent's panels, so it runs top-down on a third stream; the
    // G^< extraction of a height waits for that height's chain clusters.
    // Under stream capture (the batch graph) everything stays on st: forking
    // the plan's own stream inside a capture crashed the HIP runtime.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cap) != hipSuccess) cap = hipStreamCaptureStatusActive;
    // profiling mode 2 keeps everything on st too, so each kernel's event
    // time is its own (no overlap with the other extraction's kernels)
    const bool fork = cap == hipStreamCaptureStatusNone && !(p->profiling && p->profiling_mode == 2);
    hipStream_t sp = fork ? p->side : st;
    // the back substitution's T panels of all chain clusters, in parallel
    timed(K_CHAIN_T, 0, 0, nb, [&] { launch_chain_t(c, p->d_chainitems, p->chain_ptr[H], nb, st); });
    if (fork) {
      (void)hipEventRecord(p->ev_fork, st);
      (void)hipStreamWaitEvent(sp, p->ev_fork, 0);
      (void)hipStreamWaitEvent(p->chain, p->ev_fork, 0);
      for (int h = H; h >= 1; --h) {
        const int k0 = p->chaincl_ptr[h - 1], nck = p->chaincl_ptr[h] - k0;
        if (!nck) continue;
        timed_on(p->chain, K_CHAIN_BACK, h, 0, nb, [&] { launch_chain_back(c, p->d_chaincls + k0, nck, nb, p->chain); });
        (void)hipEventRecord(p->ev_chain[h], p->chain);
      }
    }
    for (int h = H; h >= 1; --h) {
      const int k0 = p->chaincl_ptr[h - 1], nck = p->chaincl_ptr[h] - k0;
      // the G^< source on chain clusters first: the extraction of P reads it
      if (nck) {
        if (fork) (void)hipStreamWaitEvent(sp, p->ev_chain[h], 0);
        else timed_on(sp, K_CHAIN_BACK, h, 0, nb, [&] { launch_chain_back(c, p->d_chaincls + k0, nck, nb, sp); });
      }
      for (int q = 0; q < ndg_plan::kClasses; ++q) {
        const ndg_plan::Group& g = p->groups[h * ndg_plan::kClasses + q];
        if (!g.ncl) continue;
        const int32_t* cl = p->d_levels + g.cl0;
        // the density needs only G^<, whose extraction reads none of G^r's
        // rows (its source comes from the chain kernels)
        const bool gr = mode != kRunDensity;
        if (q <= 2) {
          timed_on(sp, K_EXTRACT_SMALL_P, h, q, nb, [&] { launch_extract_small(c, cl, g.ncl, nb, g.lds, g.lds_leaf, g.size, true, sp); });
          if (gr) timed(K_EXTRACT_SMALL, h, q, nb, [&] { launch_extract_small(c, cl, g.ncl, nb, g.lds, g.lds_leaf, g.size, false, st); });
          continue;
        }
        const ColItem* ci = p->d_colitems + g.col0;
        if (g.ncol) timed_on(sp, K_DOWN_OFF_P, h, q, nb, [&] { launch_down_off(c, ci, g.ncol, nb, true, g.size, sp); });
        timed_on(sp, K_DOWN_DIAG_P, h, q, nb, [&] { launch_down_diag(c, cl, g.ncl, nb, true, g.size, sp); });
        if (gr && g.ncol) timed(K_DOWN_OFF_G, h, q, nb, [&] { launch_down_off(c, ci, g.ncol, nb, false, g.size, st); });
        if (gr) timed(K_DOWN_DIAG_G, h, q, nb, [&] { launch_down_diag(c, cl, g.ncl, nb, false, g.size, st); });
      }
    }
    if (fork) {
      (void)hipEventRecord(p->ev_join, sp);
      (void)hipStreamWaitEvent(st, p->ev_join, 0);
    }
    if (mode == kRunSolve) {
      timed(K_EPILOGUE, 0, 0, nb, [&] {
        launch_epilogue(c, nb, reinterpret_cast<double2*>(dgr), reinterpret_cast<double2*>(dgl),
                        reinterpret_cast<double2*>(dgg), st);
      });
      if (current) launch_current(c, p->d_caddr, nb, current, st);
      // further G^< passes over the same factors with other sources (the
      // G^< fronts are overwritten; the G^< diagonal was written above):
      // Sigma^> for G^> in its own step, then -i Gamma_1 for the
      // transmission.  All on st.
      for (int pass = 0; pass < 2; ++pass) {
        if (pass == 0 ? !dgg_explicit : !transmission) continue;
        launch_form_source(c, p->d_src[0], p->d_src[1], pass, nb, st);
        Ctx c2 = c;
        for (int q = 0; q < 2; ++q) c2.sig_l[q] = p->d_src[q];
        c2.sl_e0 = e0;
        launch_chain_t(c2, p->d_chainitems, p->chain_ptr[H], nb, st);
        for (int h = H; h >= 1; --h) {
          const int k0 = p->chaincl_ptr[h - 1], nck = p->chaincl_ptr[h] - k0;
          if (nck) launch_chain_back(c2, p->d_chaincls + k0, nck, nb, st);
          for (int q = 0; q < ndg_plan::kClasses; ++q) {
            const ndg_plan::Group& g = p->groups[h * ndg_plan::kClasses + q];
            if (!g.ncl) continue;
            const int32_t* cl = p->d_levels + g.cl0;
            if (q <= 2) {
              launch_extract_small(c2, cl, g.ncl, nb, g.lds, g.lds_leaf, g.size, true, st);
              continue;
            }
            if (g.ncol) launch_down_off(c2, p->d_colitems + g.col0, g.ncol, nb, true, g.size, st);
            launch_down_diag(c2, cl, g.ncl, nb, true, g.size, st);
          }
        }
        if (pass == 0) launch_epilogue_lesser(c2, nb, reinterpret_cast<double2*>(dgg_explicit), st);
        else launch_transmission(c2, p->d_caddr, nb, transmission, st);
      }
    } else
      launch_density(c, nb, cE, density, st);
    p->last_batch = nb;
  }
  if (hipGetLastError() != hipSuccess) { set_error("ndg_solve: kernel launch failed"); return NDG_EHIP; }
  return NDG_OK;
}

int symbolic_costs(const Symbolic& sy, int capacity, ndg_kernel_stat* out, int32_t* count) {
  std::vector<ClusterDesc> hd;
  layout(sy, hd);
  int ncont[2] = {0, 0};
  const int ncontacts = std::min((int)sy.contact_cluster.size(), kMaxContacts);
  for (int c = 0; c < ncontacts; ++c) ncont[c] = (int)sy.contact_pos[c].size();
  std::vector<double> fl, by;
  phonon_free_costs(sy, hd, ncont, ncontacts, fl, by);
  const int H = sy.max_height;
  int m = 0;
  for (int k = 0; k < kKernels; ++k)
    for (int h = 0; h <= H; ++h)
      for (int q = 0; q < kCostClasses; ++q) {
        const int i = cost_index(k, h, q, H);
        if (fl[i] == 0.0 && by[i] == 0.0) continue;
        if (m < capacity) {
          ndg_kernel_stat& a = out[m];
          std::memset(&a, 0, sizeof(a));
          std::snprintf(a.name, sizeof(a.name), "%s", kKernelNames[k]);
          a.height = h;
          a.size_class = q;
          a.launches = 1;
          a.flops = fl[i];
          a.bytes = by[i];
        }
        ++m;
      }
  *count = std::min(m, capacity);
  return m <= capacity ? NDG_OK : NDG_EINVAL;
}

int plan_ncontacts(const ndg_plan* p) { return p->ncontacts; }
int plan_device(const ndg_plan* p) { return p->device; }
bool plan_profiling(const ndg_plan* p) { return p->profiling; }

int plan_set_profiling(ndg_plan* p, int mode) {
  p->profiling = mode != 0;
  p->profiling_mode = mode;
  return NDG_OK;
}

int plan_profile(ndg_plan* p, int capacity, ndg_kernel_stat* out, int32_t* count) {
  if (hipSetDevice(p->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    set_error("ndg_plan_profile: device synchronisation failed");
    return NDG_EHIP;
  }
  const int H = p->max_height;
  std::vector<ndg_kernel_stat> acc((size_t)kKernels * (H + 1) * kCostClasses);
  std::memset(acc.data(), 0, sizeof(ndg_kernel_stat) * acc.size());
  for (int k = 0; k < kKernels; ++k)
    for (int h = 0; h <= H; ++h)
      for (int q = 0; q < kCostClasses; ++q) {
        ndg_kernel_stat& a = acc[cost_index(k, h, q, H)];
        std::snprintf(a.name, sizeof(a.name), "%s", kKernelNames[k]);
        a.height = h;
        a.size_class = q;
      }
  for (auto& r : p->recs) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    ndg_kernel_stat& a = acc[cost_index(r.kid, r.h, r.q, H)];
    a.launches += 1;
    a.ms += ms;
    a.flops += r.flops;
    a.bytes += r.bytes;
    p->event_pool.push_back(r.a);
    p->event_pool.push_back(r.b);
  }
  p->recs.clear();
  int m = 0;
  for (auto& a : acc)
    if (a.launches > 0 && m < capacity) out[m++] = a;
  *count = m;
  return NDG_OK;
}

int plan_status(ndg_plan* p, int32_t* code, int32_t* energy, int32_t* cluster) {
  int32_t h[4] = {0, 0, 0, 0};
  if (hipSetDevice(p->device) != hipSuccess ||
      hipMemcpy(h, p->d_status, 4 * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemset(p->d_status, 0, 4 * sizeof(int32_t)) != hipSuccess) {
    set_error("ndg_plan_status: HIP copy failed");
    return NDG_EHIP;
  }
  *code = h[0];
  *energy = h[0] ? h[1] : -1;
  *cluster = h[0] ? h[2] : -1;
  return NDG_OK;
}

int plan_export_block(ndg_plan* p, int which, int energy, int cluster, ndg_c128* out) {
  if (cluster < 0 || cluster >= p->nclusters || energy < 0 || energy >= p->last_batch || which < 0 || which > 3) {
    set_error("ndg_plan_export_block: index out of range");
    return NDG_EINVAL;
  }
  const ClusterDesc& d = p->hdesc[cluster];
  int64_t off, count;
  switch (which) {
    case 0: off = d.o_ainv; count = (int64_t)d.s * d.s; break;
    case 1: off = d.o_psi; count = (int64_t)d.s * d.b; break;
    case 2: off = d.o_fg; count = (int64_t)d.s * d.f; break;
    default: off = d.o_fp; count = (int64_t)d.s * d.f; break;
  }
  if (count == 0) return NDG_OK;
  if (hipSetDevice(p->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(out, p->d_ws + (int64_t)energy * p->stride + off, count * 16, hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("ndg_plan_export_block: HIP copy failed");
    return NDG_EHIP;
  }
  return NDG_OK;
}

}  // namespace ndg
