// Separator tree (nested dissection) and symbolic analysis -- host only.
//
// Section 3.2 organises the points of the device in clusters arranged in a
// binary tree: each separator splits its region into two parts that do not
// interact, recursively, and the clusters of one level are processed
// independently.  The partition rules (same-level clusters do not interact;
// separators small, leaves small enough to invert) are the only requirement
// on the tree; any tree obeying them gives the same Green's functions up to
// rounding.
//
// The symbolic analysis orders the points cluster by cluster in post-order
// (descendants before ancestors) and computes, for every cluster i, the set
// B_i of ancestor points coupled to the subtree of i after fill.  Only the
// blocks (i, B_i) carry nonzero Psi_{i,j} = -(A_ii)^{-1} A_ij, and the front
// of cluster i is the point list [i, B_i].
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ndg {

struct TreeOptions {
  int leaf_max = 64;     // regions with at most this many points become leaves
  int max_cluster = 64;  // clusters larger than this are split into a chain
  int kind = 0;          // 0: nested dissection, 1: layer chain, 2: contacts in the root,
                         // 3: open slab chain
  int slab = 8;          // kind 3: layers between consecutive chain separators
  int layer_max = 128;   // kind 3: separator (and end) layers up to this size stay one cluster
  const int32_t* layer_of = nullptr;  // kinds 1, 3: transport layer of every site, or null
                                      // (then layers are the sites of equal x coordinate)
};

struct Symbolic {
  int64_t n = 0;
  int nclusters = 0;
  int max_cluster = 0;      // largest s_i
  int max_boundary = 0;     // largest b_i
  int max_height = 0;
  std::vector<int32_t> perm;    // perm[new] = old site index
  std::vector<int32_t> iperm;   // iperm[old] = new index
  std::vector<int32_t> cl_off;  // cluster i owns new indices [cl_off[i], cl_off[i+1])
  std::vector<int32_t> parent;  // -1 for a root
  std::vector<std::vector<int32_t>> children;
  std::vector<int32_t> height;  // leaves 1; parent = 1 + max(children)
  std::vector<int64_t> bptr;    // B_i = bidx[bptr[i] .. bptr[i+1])
  std::vector<int32_t> bidx;    // new indices, ascending
  std::vector<int32_t> relmap;  // for each entry of bidx: position in the parent's front
  std::vector<int32_t> owner;   // owner[new index] = cluster id
  // contacts: the lowest cluster holding sites of each contact (a contact
  // larger than max_cluster spans a parent-child chain of clusters), and each
  // contact site's internal position (site order as given by the caller)
  std::vector<int32_t> contact_cluster;
  std::vector<std::vector<int32_t>> contact_pos;
  // contact self-energy entries per front: entry (a, b) of contact c goes to
  // the front of the lower of the clusters owning sites a and b, at front
  // positions (srow, scol); sflat = a * nc + b
  std::vector<int64_t> sptr;
  std::vector<int32_t> srow, scol, scid, sflat;
  // H in the new ordering, per cluster: entries of rows of cluster i whose
  // column lies in the front [i, B_i]: (local row, front column, value)
  std::vector<int64_t> hptr;
  std::vector<int32_t> hrow, hcol;
  std::vector<double> hval;
  // clusters sorted by height (ascending), level boundaries
  std::vector<int32_t> level_order;
  std::vector<int32_t> level_ptr;   // level h (1-based) -> level_order[level_ptr[h-1] .. level_ptr[h])

  int s(int i) const { return cl_off[i + 1] - cl_off[i]; }
  int b(int i) const { return (int)(bptr[i + 1] - bptr[i]); }
};

// Operation counts per energy in the convention of Section 4.1 (a product
// of i x j by j x k counts ijk, an i x i inversion counts i^3), here in
// complex multiply-adds, split by step.
struct OpCounts {
  double fold_inv = 0, fold_psi = 0, fold_update = 0;
  double gr_off = 0, gr_diag = 0;
  double gl_chain = 0, gl_off = 0, gl_diag = 0;
  double total() const {
    return fold_inv + fold_psi + fold_update + gr_off + gr_diag + gl_chain + gl_off + gl_diag;
  }
};

// Status codes mirror the C-ABI's.
enum TreeError { TREE_OK = 0, TREE_EINVAL = -1, TREE_ENOTSYM = -2, TREE_ECONTACT = -3 };

int build_symbolic(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                   int ncontacts, const int32_t* const* contact_sites, const int32_t* contact_n,
                   const double* coords, const TreeOptions& opt, Symbolic& out, std::string& err);

OpCounts count_ops(const Symbolic& sy, bool diag_only_leaves);

// RGF count for the same layered device (dense layer blocks of width w,
// nl layers), same convention: used for the complexity comparison of
// Section 4.1.
double rgf_ops(int64_t w, int64_t nl);

}  // namespace ndg
