// Nested-dissection separator tree and symbolic analysis (host only).
//
// Partition rules (Section 3.2, "Comments on the system partition"):
//   1. clusters of one level do not interact, so they are processed
//      independently;
//   2. separators are small and leaves small enough to invert.
// A contact's sites are coupled densely by its self-energy; Section 3.1
// takes Sigma^< block diagonal over clusters, so each contact lies inside one
// cluster, or, when it is larger than the largest cluster, inside one
// parent-child chain of clusters (the G^< source is then still formed along
// that chain).  With dense contact layers the tree keeps each contact as its own
// cluster below the separators (Section 3.2, Fig. 8 and the appendix, where
// the dense blocks A_11 and A_44 are leaves); variant trees give the layer
// chain of Fig. 6 (which reproduces RGF) and the contacts-in-root partition
// of Fig. 7.
#include "tree.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <functional>
#include <numeric>

namespace ndg {
namespace {

struct Builder {
  int64_t n = 0;
  const int64_t* rowptr = nullptr;
  const int32_t* col = nullptr;
  const double* coords = nullptr;
  TreeOptions opt;
  std::vector<int32_t> contact_of;                 // site -> contact id, or -1
  std::vector<std::vector<int32_t>> contacts;
  std::vector<std::vector<int32_t>> cl_pts;        // clusters, creation order
  std::vector<int32_t> cl_parent;
  std::vector<int32_t> tag;                        // region tag per site
  int tagc = 0;
  std::string err;
  bool failed = false;

  template <class F>
  void for_adj(int32_t v, F&& f) const {
    for (int64_t p = rowptr[v]; p < rowptr[v + 1]; ++p)
      if (col[p] != v) f(col[p]);
    int c = contact_of[v];
    if (c >= 0)
      for (int32_t u : contacts[c])
        if (u != v) f(u);
  }

  double x(int32_t v, int ax) const { return coords[3 * (int64_t)v + ax]; }

  std::vector<std::vector<int32_t>> components(const std::vector<int32_t>& R, int t) {
    std::vector<std::vector<int32_t>> out;
    int t2 = ++tagc;  // visited mark
    std::vector<int32_t> stack;
    for (int32_t s0 : R) {
      if (tag[s0] != t) continue;
      std::vector<int32_t> comp;
      tag[s0] = t2;
      stack.push_back(s0);
      while (!stack.empty()) {
        int32_t v = stack.back();
        stack.pop_back();
        comp.push_back(v);
        for_adj(v, [&](int32_t u) {
          if (tag[u] == t) {
            tag[u] = t2;
            stack.push_back(u);
          }
        });
      }
      out.push_back(std::move(comp));
    }
    for (int32_t v : R) tag[v] = t;
    return out;
  }

  // Adds pts as one cluster, or a chain of clusters of at most max_cluster
  // points (top of the chain first).  Returns the bottom cluster.
  int add_chain(std::vector<int32_t> pts, int parent, int maxc = 0) {
    if (maxc <= 0) maxc = opt.max_cluster;
    if (pts.empty()) return parent;
    // order points along their longest extent so chain pieces are compact
    if (coords && pts.size() > 1) {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int32_t v : pts)
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], x(v, a));
          hi[a] = std::max(hi[a], x(v, a));
        }
      int ax = 0;
      for (int a = 1; a < 3; ++a)
        if (hi[a] - lo[a] > hi[ax] - lo[ax]) ax = a;
      std::stable_sort(pts.begin(), pts.end(), [&](int32_t p, int32_t q) {
        double xp = x(p, ax), xq = x(q, ax);
        return xp < xq || (xp == xq && p < q);
      });
    } else {
      std::sort(pts.begin(), pts.end());
    }
    int nchunk = (int)((pts.size() + maxc - 1) / maxc);
    int cur = parent;
    for (int k = nchunk - 1; k >= 0; --k) {  // top of chain = last chunk
      size_t a = pts.size() * k / nchunk, b = pts.size() * (k + 1) / nchunk;
      std::vector<int32_t> c(pts.begin() + a, pts.begin() + b);
      std::sort(c.begin(), c.end());
      cl_pts.push_back(std::move(c));
      cl_parent.push_back(cur);
      cur = (int)cl_pts.size() - 1;
    }
    return cur;
  }

  // Contacts fully inside the region tagged t.
  std::vector<int> contacts_in(int t) const {
    std::vector<int> out;
    for (int c = 0; c < (int)contacts.size(); ++c)
      if (!contacts[c].empty() && tag[contacts[c][0]] == t) out.push_back(c);
    return out;
  }

  // Vertex separator from a coordinate cut: left = {x <= m}, right = {x > m},
  // S = left vertices with a neighbour on the right.  Returns false when no
  // axis gives a cut that keeps every contact inside one of S, left \ S, right.
  bool geometric_cut(const std::vector<int32_t>& R, int t, const std::vector<int>& cin,
                     std::vector<int32_t>& S) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v : R)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], x(v, a));
        hi[a] = std::max(hi[a], x(v, a));
      }
    int axes[3] = {0, 1, 2};
    std::sort(axes, axes + 3, [&](int p, int q) { return hi[p] - lo[p] > hi[q] - lo[q]; });
    std::vector<double> vals(R.size());
    for (int ai = 0; ai < 3; ++ai) {
      int ax = axes[ai];
      double ext = hi[ax] - lo[ax];
      if (ext <= 1e-12) break;
      double eps = 1e-9 * std::max(1.0, ext);
      for (size_t k = 0; k < R.size(); ++k) vals[k] = x(R[k], ax);
      std::vector<double> sv = vals;
      size_t mid = (sv.size() - 1) / 2;
      std::nth_element(sv.begin(), sv.begin() + mid, sv.end());
      double m = sv[mid];
      if (m >= hi[ax] - eps) continue;
      int t2 = ++tagc;  // mark right side
      std::vector<int32_t> cand;
      for (size_t k = 0; k < R.size(); ++k)
        if (vals[k] > m + eps) tag[R[k]] = t2;
      S.clear();
      for (size_t k = 0; k < R.size(); ++k) {
        if (vals[k] > m + eps) continue;
        bool sep = false;
        for_adj(R[k], [&](int32_t u) { sep |= (tag[u] == t2); });
        if (sep) S.push_back(R[k]);
      }
      for (size_t k = 0; k < R.size(); ++k) tag[R[k]] = t;
      // contact safety
      bool safe = !S.empty() && S.size() < R.size();
      if (safe) {
        int t3 = ++tagc;
        for (int32_t v : S) tag[v] = t3;
        for (int c : cin) {
          size_t inS = 0, inRight = 0;
          for (int32_t v : contacts[c]) {
            if (tag[v] == t3) ++inS;
            else if (x(v, ax) > m + eps) ++inRight;
          }
          size_t sz = contacts[c].size();
          bool whole = (inS == sz) || (inRight == sz) || (inS == 0 && inRight == 0);
          if (!whole) safe = false;
        }
        for (int32_t v : S) tag[v] = t;
      }
      if (safe) return true;
    }
    S.clear();
    return false;
  }

  // Level-set separator from a pseudo-peripheral vertex (used without
  // coordinates).
  bool bfs_cut(const std::vector<int32_t>& R, int t, const std::vector<int>& cin,
               std::vector<int32_t>& S) {
    auto levels_from = [&](int32_t s0, std::vector<std::vector<int32_t>>& lev) {
      lev.clear();
      int t2 = ++tagc;
      std::vector<int32_t> cur{s0};
      tag[s0] = t2;
      while (!cur.empty()) {
        lev.push_back(cur);
        std::vector<int32_t> nxt;
        for (int32_t v : cur)
          for_adj(v, [&](int32_t u) {
            if (tag[u] == t) {
              tag[u] = t2;
              nxt.push_back(u);
            }
          });
        cur.swap(nxt);
      }
      for (int32_t v : R) tag[v] = t;
    };
    std::vector<std::vector<int32_t>> lev;
    int32_t s0 = R[0];
    for (int it = 0; it < 3; ++it) {
      levels_from(s0, lev);
      const auto& last = lev.back();
      s0 = *std::min_element(last.begin(), last.end());
    }
    levels_from(s0, lev);
    if (lev.size() < 3) return false;
    size_t half = R.size() / 2, acc = 0;
    int best = -1;
    for (int L = 0; L < (int)lev.size(); ++L) {
      acc += lev[L].size();
      if (acc >= half) { best = L; break; }
    }
    best = std::max(1, std::min(best, (int)lev.size() - 2));
    for (int d = 0; d < (int)lev.size(); ++d) {
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int L = best + sgn * d;
        if (L < 1 || L > (int)lev.size() - 2) continue;
        S = lev[L];
        int t3 = ++tagc;
        for (int32_t v : S) tag[v] = t3;
        bool safe = true;
        for (int c : cin) {
          size_t inS = 0;
          for (int32_t v : contacts[c]) inS += (tag[v] == t3);
          if (inS != 0 && inS != contacts[c].size()) safe = false;
        }
        for (int32_t v : S) tag[v] = t;
        if (safe) return true;
        if (d == 0) break;
      }
    }
    S.clear();
    return false;
  }

  void nd(std::vector<int32_t> R, int parent, int depth) {
    if (R.empty() || failed) return;
    if (depth > 4096) { err = "separator tree too deep"; failed = true; return; }
    int t = ++tagc;
    for (int32_t v : R) tag[v] = t;
    auto comps = components(R, t);
    if (comps.size() > 1) {
      for (auto& c : comps) nd(std::move(c), parent, depth + 1);
      return;
    }
    std::vector<int> cin = contacts_in(t);
    bool only_contact = cin.size() == 1 && contacts[cin[0]].size() == R.size();
    if ((int)R.size() <= opt.leaf_max || only_contact) {
      add_chain(R, parent);
      return;
    }
    std::vector<int32_t> S;
    bool small = (int64_t)R.size() <= 4 * (int64_t)opt.leaf_max;
    bool ok = false;
    if (!(small && !cin.empty())) ok = coords ? geometric_cut(R, t, cin, S) : bfs_cut(R, t, cin, S);
    if (!ok && !cin.empty()) {
      // peel the contact: separator = its neighbours in the region
      const auto& C = contacts[cin[0]];
      int tc = ++tagc;
      for (int32_t v : C) tag[v] = tc;
      int ts = ++tagc;
      S.clear();
      for (int32_t v : C)
        for_adj(v, [&](int32_t u) {
          if (tag[u] == t) {
            tag[u] = ts;
            S.push_back(u);
          }
        });
      std::vector<int32_t> rest;
      for (int32_t v : R)
        if (tag[v] == t) rest.push_back(v);
      for (int32_t v : R) tag[v] = t;
      int bottom = add_chain(S, parent);
      add_chain(C, bottom);
      nd(std::move(rest), bottom, depth + 1);
      return;
    }
    if (!ok) {  // no separator found: keep the region whole
      add_chain(R, parent);
      return;
    }
    int ts = ++tagc;
    for (int32_t v : S) tag[v] = ts;
    std::vector<int32_t> rest;
    for (int32_t v : R)
      if (tag[v] == t) rest.push_back(v);
    for (int32_t v : R) tag[v] = t;
    int bottom = add_chain(S, parent);
    nd(std::move(rest), bottom, depth + 1);  // splits into components below
  }
};

}  // namespace

int build_symbolic(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                   int ncontacts, const int32_t* const* contact_sites, const int32_t* contact_n,
                   const double* coords, const TreeOptions& opt, Symbolic& out, std::string& err) {
  out = Symbolic();
  if (n <= 0 || !rowptr || !col || !val) { err = "empty or null H"; return TREE_EINVAL; }
  if (opt.leaf_max < 1 || opt.max_cluster < 1 || opt.kind < 0 || opt.kind > 3 || opt.slab < 0) {
    err = "bad tree options";
    return TREE_EINVAL;
  }
  if (rowptr[0] != 0) { err = "rowptr[0] must be 0"; return TREE_EINVAL; }
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) { err = "rowptr not monotone"; return TREE_EINVAL; }
  for (int64_t p = 0; p < rowptr[n]; ++p)
    if (col[p] < 0 || col[p] >= n) { err = "column index out of range"; return TREE_EINVAL; }
  // symmetry of H (pattern and values)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      int32_t j = col[p];
      bool found = false;
      for (int64_t q = rowptr[j]; q < rowptr[j + 1]; ++q)
        if (col[q] == i) { found = std::fabs(val[q] - val[p]) <= 1e-13 * (std::fabs(val[p]) + 1e-300) || val[q] == val[p]; break; }
      if (!found) { err = "H is not symmetric"; return TREE_ENOTSYM; }
    }
  Builder B;
  B.n = n; B.rowptr = rowptr; B.col = col; B.coords = coords; B.opt = opt;
  B.contact_of.assign(n, -1);
  B.tag.assign(n, 0);
  for (int c = 0; c < ncontacts; ++c) {
    if (contact_n[c] <= 0 || !contact_sites[c]) { err = "empty contact"; return TREE_EINVAL; }
    std::vector<int32_t> s(contact_sites[c], contact_sites[c] + contact_n[c]);
    for (int32_t v : s) {
      if (v < 0 || v >= n) { err = "contact site out of range"; return TREE_EINVAL; }
      if (B.contact_of[v] >= 0) { err = "contacts overlap or repeat a site"; return TREE_ECONTACT; }
      B.contact_of[v] = c;
    }
    B.contacts.push_back(s);
  }
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  if (opt.kind == 0) {
    B.nd(all, -1, 0);
  } else if (opt.kind == 1 || opt.kind == 3) {
    // transport layers: the caller's layer index per site, else the sites of
    // equal transport (x) coordinate
    std::vector<std::vector<int32_t>> layers;
    if (opt.layer_of) {
      std::vector<int32_t> idx(all);
      for (int32_t v : idx)
        if (opt.layer_of[v] < 0) { err = "negative layer index"; return TREE_EINVAL; }
      std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return opt.layer_of[a] < opt.layer_of[b]; });
      for (size_t k = 0; k < idx.size(); ++k) {
        if (k == 0 || opt.layer_of[idx[k]] != opt.layer_of[idx[k - 1]]) layers.emplace_back();
        layers.back().push_back(idx[k]);
      }
    } else if (coords) {
      std::vector<int32_t> idx(all);
      std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return coords[3 * (int64_t)a] < coords[3 * (int64_t)b]; });
      for (size_t k = 0; k < idx.size(); ++k) {
        if (k == 0 || coords[3 * (int64_t)idx[k]] > coords[3 * (int64_t)idx[k - 1]] + 1e-9) layers.emplace_back();
        layers.back().push_back(idx[k]);
      }
    } else {
      err = "the layer-chain trees need coordinates or a layer index per site";
      return TREE_EINVAL;
    }
    // merge layers holding pieces of one contact
    for (int c = 0; c < ncontacts; ++c) {
      std::vector<int> hit;
      for (int L = 0; L < (int)layers.size(); ++L)
        for (int32_t v : layers[L])
          if (B.contact_of[v] == c) { hit.push_back(L); break; }
      for (size_t k = 1; k < hit.size(); ++k) {
        for (int L = hit[0] + 1; L <= hit[k]; ++L) {
          layers[hit[0]].insert(layers[hit[0]].end(), layers[L].begin(), layers[L].end());
          layers[L].clear();
        }
      }
    }
    layers.erase(std::remove_if(layers.begin(), layers.end(), [](const std::vector<int32_t>& L) { return L.empty(); }),
                 layers.end());
    // the slab chain needs every coupling to join equal or consecutive
    // layers (block tridiagonal), or a slab would reach past its separators
    if (opt.kind == 3) {
      std::vector<int32_t> lid(n, -1);
      for (int L = 0; L < (int)layers.size(); ++L)
        for (int32_t v : layers[L]) lid[v] = L;
      for (int64_t i = 0; i < n; ++i) {
        bool bad = false;
        B.for_adj((int32_t)i, [&](int32_t u) { bad |= std::abs(lid[u] - lid[i]) > 1; });
        if (bad) { err = "the layers do not make H block tridiagonal"; return TREE_EINVAL; }
      }
    }
    if (opt.kind == 1) {
      int cur = -1;
      for (int L = (int)layers.size() - 1; L >= 0; --L) cur = B.add_chain(layers[L], cur);
    } else {
      // open slab chain: separator layers every slab + 1 layers, chained from
      // the middle layer (the root) towards both end layers; the slabs of
      // layers between two separators hang below the lower of the two and are
      // dissected as above.  Every chain cluster's subtree then holds an end
      // layer, so the region it folds is open through that end's contact.
      const int m = (int)layers.size(), step = opt.slab + 1, r = m / 2;
      auto interior = [&](int a, int b) {  // layers strictly between a and b
        std::vector<int32_t> R;
        for (int L = a + 1; L < b; ++L) R.insert(R.end(), layers[L].begin(), layers[L].end());
        return R;
      };
      // a layer is kept whole up to layer_max points (one cluster per chain
      // level: fewer levels and taller matrix-core tiles); a wider one is
      // split into a parent-child chain of clusters
      const int lmax = opt.layer_max;
      const int root = B.add_chain(layers[r], -1, lmax);
      for (int side = -1; side <= 1; side += 2) {
        if ((side < 0 && r == 0) || (side > 0 && r == m - 1)) continue;
        int up = r, up_cl = root;
        while (true) {
          int nxt = up + side * step;
          const bool end = side < 0 ? nxt <= 0 : nxt >= m - 1;
          if (end) nxt = side < 0 ? 0 : m - 1;
          const int cl = B.add_chain(layers[nxt], up_cl, lmax);
          // the slab between this separator and the one above it
          B.nd(side < 0 ? interior(nxt, up) : interior(up, nxt), cl, 1);
          if (end) break;
          up = nxt;
          up_cl = cl;
        }
        if (B.failed) break;
      }
    }
  } else {
    // contacts merged into the top of the tree, nested dissection below
    int cur = -1;
    for (int c = ncontacts - 1; c >= 0; --c) cur = B.add_chain(B.contacts[c], cur);
    std::vector<int32_t> rest;
    for (int32_t v : all)
      if (B.contact_of[v] < 0) rest.push_back(v);
    std::vector<std::vector<int32_t>> saved = B.contacts;
    std::fill(B.contact_of.begin(), B.contact_of.end(), -1);
    B.contacts.clear();
    B.nd(rest, cur, 0);
    B.contacts = saved;
    for (int c = 0; c < ncontacts; ++c)
      for (int32_t v : saved[c]) B.contact_of[v] = c;
  }
  if (B.failed) { err = B.err; return TREE_ECONTACT; }

  // ---- post-order numbering -------------------------------------------
  const int nc = (int)B.cl_pts.size();
  std::vector<std::vector<int32_t>> kids(nc);
  std::vector<int32_t> roots;
  for (int c = 0; c < nc; ++c) {
    if (B.cl_parent[c] < 0) roots.push_back(c);
    else kids[B.cl_parent[c]].push_back(c);
  }
  std::vector<int32_t> post;  // post[new id] = creation id
  post.reserve(nc);
  {
    std::vector<std::pair<int32_t, size_t>> st;
    for (int32_t r : roots) {
      st.push_back({r, 0});
      while (!st.empty()) {
        auto& top = st.back();
        if (top.second < kids[top.first].size()) {
          int32_t ch = kids[top.first][top.second++];
          st.push_back({ch, 0});
        } else {
          post.push_back(top.first);
          st.pop_back();
        }
      }
    }
  }
  std::vector<int32_t> newid(nc);
  for (int k = 0; k < nc; ++k) newid[post[k]] = k;
  Symbolic& sy = out;
  sy.n = n;
  sy.nclusters = nc;
  sy.cl_off.assign(nc + 1, 0);
  sy.parent.assign(nc, -1);
  sy.children.assign(nc, {});
  for (int k = 0; k < nc; ++k) {
    int c = post[k];
    sy.cl_off[k + 1] = sy.cl_off[k] + (int32_t)B.cl_pts[c].size();
    sy.parent[k] = B.cl_parent[c] < 0 ? -1 : newid[B.cl_parent[c]];
  }
  for (int k = 0; k < nc; ++k)
    if (sy.parent[k] >= 0) sy.children[sy.parent[k]].push_back(k);
  if (sy.cl_off[nc] != n) { err = "internal: clusters do not cover all sites"; return TREE_EINVAL; }
  sy.perm.assign(n, -1);
  sy.iperm.assign(n, -1);
  sy.owner.assign(n, -1);
  for (int k = 0; k < nc; ++k) {
    const auto& pts = B.cl_pts[post[k]];
    for (size_t q = 0; q < pts.size(); ++q) {
      int32_t nw = sy.cl_off[k] + (int32_t)q;
      if (sy.iperm[pts[q]] >= 0) { err = "internal: site in two clusters"; return TREE_EINVAL; }
      sy.perm[nw] = pts[q];
      sy.iperm[pts[q]] = nw;
      sy.owner[nw] = k;
    }
  }
  // subtree interval [sub_lo, cl_off[k+1])
  std::vector<int32_t> sub_lo(nc);
  for (int k = 0; k < nc; ++k) {
    sub_lo[k] = sy.cl_off[k];
    for (int32_t ch : sy.children[k]) sub_lo[k] = std::min(sub_lo[k], sub_lo[ch]);
  }
  auto is_ancestor = [&](int a, int k) {  // a is a strict ancestor of k
    return a != k && sub_lo[a] <= sub_lo[k] && sy.cl_off[k + 1] <= sy.cl_off[a + 1];
  };
  sy.height.assign(nc, 1);
  for (int k = 0; k < nc; ++k)
    for (int32_t ch : sy.children[k]) sy.height[k] = std::max(sy.height[k], sy.height[ch] + 1);
  // ---- boundary sets B_i (post-order, children first) ----------------
  std::vector<std::vector<int32_t>> Bs(nc);
  for (int k = 0; k < nc; ++k) {
    std::vector<int32_t> acc;
    int32_t hiI = sy.cl_off[k + 1];
    for (int32_t nw = sy.cl_off[k]; nw < hiI; ++nw) {
      int32_t v = sy.perm[nw];
      bool bad = false;
      B.for_adj(v, [&](int32_t u) {
        int32_t un = sy.iperm[u];
        if (un >= sub_lo[k] && un < hiI) return;  // inside the subtree
        if (!is_ancestor(sy.owner[un], k)) bad = true;
        else acc.push_back(un);
      });
      if (bad) { err = "partition violates the separator rule (edge between unrelated clusters)"; return TREE_EINVAL; }
    }
    for (int32_t ch : sy.children[k])
      for (int32_t u : Bs[ch])
        if (u >= hiI) acc.push_back(u);
    std::sort(acc.begin(), acc.end());
    acc.erase(std::unique(acc.begin(), acc.end()), acc.end());
    Bs[k] = std::move(acc);
    if (sy.parent[k] < 0 && !Bs[k].empty()) { err = "internal: root with a boundary"; return TREE_EINVAL; }
  }
  sy.bptr.assign(nc + 1, 0);
  for (int k = 0; k < nc; ++k) sy.bptr[k + 1] = sy.bptr[k] + (int64_t)Bs[k].size();
  sy.bidx.resize(sy.bptr[nc]);
  sy.relmap.resize(sy.bptr[nc]);
  for (int k = 0; k < nc; ++k) {
    std::copy(Bs[k].begin(), Bs[k].end(), sy.bidx.begin() + sy.bptr[k]);
    int p = sy.parent[k];
    for (size_t q = 0; q < Bs[k].size(); ++q) {
      int32_t u = Bs[k][q];
      int32_t pos;
      if (u >= sy.cl_off[p] && u < sy.cl_off[p + 1]) pos = u - sy.cl_off[p];
      else {
        auto it = std::lower_bound(Bs[p].begin(), Bs[p].end(), u);
        if (it == Bs[p].end() || *it != u) { err = "internal: boundary not inside the parent's front"; return TREE_EINVAL; }
        pos = sy.s(p) + (int32_t)(it - Bs[p].begin());
      }
      sy.relmap[sy.bptr[k] + q] = pos;
    }
  }
  // ---- H entries per front ----------------------------------------------
  sy.hptr.assign(nc + 1, 0);
  for (int k = 0; k < nc; ++k) {
    int32_t lo = sy.cl_off[k], hiI = sy.cl_off[k + 1];
    const auto& Bk = Bs[k];
    for (int32_t nw = lo; nw < hiI; ++nw) {
      int32_t v = sy.perm[nw];
      for (int64_t p = rowptr[v]; p < rowptr[v + 1]; ++p) {
        int32_t un = sy.iperm[col[p]];
        int32_t fc;
        if (un >= lo && un < hiI) fc = un - lo;
        else {
          auto it = std::lower_bound(Bk.begin(), Bk.end(), un);
          if (it == Bk.end() || *it != un) continue;  // belongs to a descendant's front
          fc = (hiI - lo) + (int32_t)(it - Bk.begin());
        }
        sy.hrow.push_back(nw - lo);
        sy.hcol.push_back(fc);
        sy.hval.push_back(val[p]);
      }
    }
    sy.hptr[k + 1] = (int64_t)sy.hrow.size();
  }
  // ---- contacts -----------------------------------------------------------
  // A contact lies in one cluster, or (when larger than max_cluster) in a
  // parent-child chain of clusters; its self-energy entries are placed in the
  // front of the lower cluster of each pair.
  auto front_pos = [&](int k, int32_t nw) -> int32_t {
    if (nw >= sy.cl_off[k] && nw < sy.cl_off[k + 1]) return nw - sy.cl_off[k];
    auto b0 = sy.bidx.begin() + sy.bptr[k], b1 = sy.bidx.begin() + sy.bptr[k + 1];
    auto it = std::lower_bound(b0, b1, nw);
    if (it == b1 || *it != nw) return -1;
    return sy.s(k) + (int32_t)(it - b0);
  };
  std::vector<std::vector<std::array<int32_t, 4>>> sent(nc);
  for (int c = 0; c < ncontacts; ++c) {
    const auto& cs = B.contacts[c];
    const int ncs = (int)cs.size();
    std::vector<int32_t> pos(ncs), own(ncs);
    int low = nc;
    for (int a = 0; a < ncs; ++a) {
      pos[a] = sy.iperm[cs[a]];
      own[a] = sy.owner[pos[a]];
      low = std::min(low, own[a]);
    }
    for (int a = 0; a < ncs; ++a)
      if (own[a] != low && !is_ancestor(own[a], low)) { err = "contact split across unrelated clusters"; return TREE_ECONTACT; }
    for (int a = 0; a < ncs; ++a)
      for (int b = 0; b < ncs; ++b) {
        const int k = std::min(own[a], own[b]);  // post-order: the lower cluster has the smaller id
        const int32_t r = front_pos(k, pos[a]), q = front_pos(k, pos[b]);
        if (r < 0 || q < 0) { err = "internal: contact coupling outside a front"; return TREE_EINVAL; }
        sent[k].push_back({r, q, c, a * ncs + b});
      }
    sy.contact_cluster.push_back(low);
    sy.contact_pos.push_back(pos);
  }
  sy.sptr.assign(nc + 1, 0);
  for (int k = 0; k < nc; ++k) {
    for (const auto& en : sent[k]) {
      sy.srow.push_back(en[0]);
      sy.scol.push_back(en[1]);
      sy.scid.push_back(en[2]);
      sy.sflat.push_back(en[3]);
    }
    sy.sptr[k + 1] = (int64_t)sy.srow.size();
  }
  // ---- levels ---------------------------------------------------------------
  sy.max_height = 0;
  for (int k = 0; k < nc; ++k) sy.max_height = std::max(sy.max_height, sy.height[k]);
  sy.level_ptr.assign(sy.max_height + 1, 0);
  for (int k = 0; k < nc; ++k) sy.level_ptr[sy.height[k]]++;
  for (int h = 1; h <= sy.max_height; ++h) sy.level_ptr[h] += sy.level_ptr[h - 1];
  sy.level_order.resize(nc);
  {
    std::vector<int32_t> pos(sy.level_ptr.begin(), sy.level_ptr.end() - 1);
    for (int k = 0; k < nc; ++k) sy.level_order[pos[sy.height[k] - 1]++] = k;
  }
  sy.max_cluster = 0;
  sy.max_boundary = 0;
  for (int k = 0; k < nc; ++k) {
    sy.max_cluster = std::max(sy.max_cluster, sy.s(k));
    sy.max_boundary = std::max(sy.max_boundary, sy.b(k));
  }
  return TREE_OK;
}

OpCounts count_ops(const Symbolic& sy, bool diag_only_leaves) {
  OpCounts oc;
  // a leaf forms only the diagonal of its own block when nobody reads the
  // rest: its front fits one on-chip block (s + b <= 64) and it does not lie
  // on a contact's chain (those keep their rows for the G^< source)
  std::vector<char> on_chain(sy.nclusters, 0);
  for (int32_t c0 : sy.contact_cluster)
    for (int k = c0; k >= 0; k = sy.parent[k]) on_chain[k] = 1;
  for (int k = 0; k < sy.nclusters; ++k) {
    double s = sy.s(k), b = sy.b(k);
    bool leaf = sy.children[k].empty() && s + b <= 64 && !on_chain[k];
    oc.fold_inv += s * s * s;
    oc.fold_psi += s * s * b;
    oc.fold_update += s * b * b;
    oc.gr_off += s * b * b;
    oc.gl_off += s * b * b;
    double d = (leaf && diag_only_leaves) ? s * b : s * s * b;
    oc.gr_diag += d;
    oc.gl_diag += d;
  }
  for (size_t c = 0; c < sy.contact_cluster.size(); ++c) {
    double sc = (double)sy.contact_pos[c].size();
    for (int k = sy.contact_cluster[c]; k >= 0; k = sy.parent[k]) {
      double s = sy.s(k), b = sy.b(k);
      // forward substitution, D^{-1}, back substitution, W and initial P
      oc.gl_chain += s * b * sc + s * s * sc + s * b * sc + s * sc * sc + s * sc * (s + b);
    }
  }
  return oc;
}

double rgf_ops(int64_t w, int64_t nl) {
  // per layer: fold 2 products + 1 inversion; extract 4 products (G^r);
  // lesser fold 4 products, lesser extract 7 products
  double w3 = (double)w * w * w;
  return (3.0 + 4.0 + 4.0 + 7.0) * w3 * (double)nl;
}

}  // namespace ndg
