// Device-side data layout shared by the runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ndg {

// Per-cluster descriptor (device).  Offsets are in complex elements inside
// one energy's slab of the workspace; -1 when a block does not exist.
struct ClusterDesc {
  int64_t o_ainv;   // s x s   pivot-block inverse (A_ii^(fold))^{-1}
  int64_t o_psi;    // s x b   Psi_{i,B_i} = -A_ii^{-1} A_{i,B_i}
  int64_t o_upd;    // b x b   Schur contribution passed to the parent front
  int64_t o_fg;     // s x f   rows of cluster i of the front [i, B_i]: the assembled rows of A
                    //         during the fold, then [G_ii, G_{i,B}] after the extraction
  int64_t o_fp;     // s x f   [G^<_ii, G^<_{i,B}] (the source term before the extraction)
  int64_t o_zf[2];  // f x sc  per contact on whose chain the cluster lies: forward solve
  int64_t o_xf[2];  // f x sc  per contact: rows of the contact's column of G^r over the front
  int64_t o_t[2];   // s x sc  per contact: scratch
  int32_t s, b, f, parent;
  int32_t pt_off;   // first internal position of the cluster
  int32_t bptr;     // B_i / relmap entries start here
  int32_t hptr0, hptr1;
  int32_t sptr0, sptr1;   // contact self-energy entries of this front
  int32_t chain_child[2]; // per contact: child on the contact's chain, -1 if none
  int32_t chain_mask;     // bit c: the cluster is on contact c's chain
  // front assembly: the cluster's rows of -H over the front (s x f,
  // mirrored for the B rows), the contact self-energy index map (f x f,
  // (contact << 24) | flat index, -1 where none; -1 offset if the front has
  // no entries), and the parent's front positions -> index in this
  // cluster's B (f_parent entries, -1 where absent; -1 offset for a root)
  int64_t o_hf, o_smap, o_pinv;
  // extraction gather: slab offsets of the entries of X_{B,B} (b x b int32,
  // see Ctx::gaddr)
  int64_t o_gaddr;
  // when B is a run of consecutive points of one ancestor (a contact chain's
  // separator under its parent layer): X_{B,B} is a dense block of that
  // ancestor's stored G^r rows, at o_bbd with row stride bbd_ld (-1: use the
  // gather table)
  int64_t o_bbd;
  // leading entries of B owned by the parent (B is sorted and the parent's
  // points precede its ancestors'): the rows of the contribution that land in
  // the parent's own rows
  int32_t nself, bbd_ld;
};

// Per site in the caller's order: slab offsets of its diagonal entries in
// the G^r and G^< fronts, and its cluster.
struct SiteDiag { int64_t og, ol; int32_t cl, pad; };

struct UpdItem { int32_t cl, tr, tc, pad; };   // Schur update tile (rows tr*TM.., cols tc*64..)
struct ColItem { int32_t cl, tc; };            // column tile of an s x b panel
struct ChainItem { int32_t cl, c; };           // chain cluster and contact

struct Ctx {
  const ClusterDesc* cl;
  const int32_t* relmap;
  const int32_t* kids_ptr;   // per cluster: [kids_ptr[i], kids_ptr[i+1]) into kids
  const int32_t* kids;
  const int32_t* hrow;
  const int32_t* hcol;
  const double* hval;
  const int32_t* perm;
  const int32_t* owner;
  const int32_t* cpos[2];    // contact site a -> internal position
  const int32_t* srow;       // contact self-energy entries per front
  const int32_t* scol;
  const int32_t* scid;
  const int32_t* sflat;
  const double* hfront;      // see ClusterDesc::o_hf
  const int32_t* smap;       // see ClusterDesc::o_smap
  const int32_t* pinv;       // see ClusterDesc::o_pinv
  // per cluster (ClusterDesc::o_gaddr), entry (u, v) of X_{B,B}: the slab
  // offset of G^r(B[u], B[v]) in the stored rows of the lower owning
  // cluster, bit 31 set when it is stored as G^r(B[v], B[u]); the G^< fronts
  // lie pdelta entries after the G^r fronts
  const int32_t* gaddr;
  int64_t pdelta;
  const SiteDiag* sdiag;     // [n], caller's site order
  int32_t nc[2];
  int32_t ncontacts;
  int32_t n;
  double2* ws;
  int64_t stride;            // complex elements per energy slab
  const double* E;
  int32_t e0;                // first energy of the batch
  const int32_t* e0p;        // if set, the batch starts at e0 + *e0p (advanced between graph replays)
  int32_t nE;                // energies in E: batch slots at or beyond it are skipped
  double eta;
  const double* V;           // may be null
  const double2* sig_r[2];
  const double2* sig_l[2];
  int32_t sl_e0;             // energy index of sig_l[c][0] (0: the caller's arrays; the batch
                             // start when sig_l points at the library's per-batch sources)
  // diagonal phonon self-energies, [nE][n] in the caller's site order, or
  // null: Sigma^r_ph enters A's diagonal; with scat set, every cluster's
  // G^< source comes from the all-ancestor N fold (Sigma^<_ph) and the
  // contact chains
  const double2* sig_r_ph;
  const double2* sig_l_ph;
  int32_t scat;
  int32_t* status;           // [code, energy, cluster]
  double* growth;            // [nE] or null: max over clusters of ||A_ii^{-1}|| ||A_iB||
  int32_t mixed;             // 1: Schur updates and extraction products on FP32 matrix cores
};

// Multi-right-hand-side solves with the factors of the fold (adjoint).
struct RhsCtx {
  // right-hand side (the columns of all contacts side by side), formed where
  // the forward substitution reads it: ymode 0 the unit columns E_c
  // (cinv[row] = the column of a contact site, or -1), ymode 1
  // Lambda conj(G_{:,c}) from Gc and nbar
  int32_t ymode;
  const int32_t* cinv;
  double2* X;         // [nb][n][m] solutions
  double2* Gc;        // [nb][n][m] contact columns of G^r
  double2* Z;         // [nb][zstride] per-cluster front vectors (f x m)
  const int64_t* o_vec;  // per-cluster offset into a Z slab
  int64_t zstride;
  int32_t n, m;
  const int32_t* bidx;   // B_i as internal positions
  const double* nbar;    // cotangent of the density (caller order)
  double* part;          // [nb][n] per-energy partial gradients
};

// All-ancestor rows for a Sigma^< on every cluster (diagonal phonon
// self-energy).  Cluster i's frame lists its own points, then those of its
// ancestors, parent first (ascending internal positions); its width is
// g_i = s_i + W_i with W_i the number of ancestor points.  The ancestors'
// frames are tails of this one: ancestor a's frame starts at column
// ao_i[a] of i's.
struct ScatDesc {
  int64_t o_g;     // s x g block of the scattering slab: the rows [G_ii, G_{i,Anc}]
                   // of the paper's G^(0), overwritten in place by N_i
  int32_t g;       // frame width s + W
  int32_t D;       // number of ancestors
  int32_t tab;     // into ScatCtx::atab: D + 1 cluster ids (the cluster, its
                   // ancestors parent first), then the D + 2 frame offsets ao
  int32_t lk0, lk1;  // descendants whose B meets this cluster: ScatCtx::lk[lk0 .. lk1)
  int32_t pad;
};
// descendant d whose B contains points of the cluster: umap[map .. map + s)
// gives, per point of the cluster, its index in B_d (or -1); col is the
// column of the cluster's frame inside d's frame
struct LkItem { int32_t d, map, col, pad; };
// per entry of B_i (indexed like relmap): its column in i's frame and the
// index in i's chain of the cluster that owns it
struct BPos { int32_t col, a; };

struct ScatCtx {
  const ScatDesc* sd;
  const int32_t* atab;
  const BPos* bpos;
  const LkItem* lk;
  const int32_t* umap;
  double2* ws;       // [nb][stride]
  int64_t stride;
};
constexpr int kMaxAncestors = 63;
constexpr int kClusterRows = 64;  // largest cluster the kernels hold per block
// tile_rows 16, 32 or 64 (at least the largest cluster of the launch);
// leaves: the launch holds only leaves (height 1), which store their N
void launch_anc_g(const Ctx& c, const ScatCtx& x, const ColItem* it, int nit, int nb, int tile_rows,
                  bool leaves, hipStream_t st);
void launch_anc_n(const Ctx& c, const ScatCtx& x, const ColItem* it, int nit, int nb, int tile_rows,
                  hipStream_t st);
void launch_anc_p0(const Ctx& c, const ScatCtx& x, const int32_t* cls, int ncl, int nb, int tile_rows,
                   hipStream_t st);
// self-consistent Born update over count = nE n entries: S' = d0 diag G,
// S <- (1 - mix) S + mix S' for Sigma^r_ph and Sigma^<_ph; out[0] = max
// |S' - S|, out[1] = max |S'| (part: kScbaBlocks x 2 doubles of scratch)
constexpr int kScbaBlocks = 1024;
// terminal current spectral density per contact and energy of the batch,
// cur[(e0 + e) * ncontacts + c] (caddr: see the plan's contact tables)
void launch_current(const Ctx& c, const int32_t* caddr, int nb, double* cur, hipStream_t st);
// Sources of the extra G^< passes, per energy of the batch and contact
// ([nb][nc][nc] each): which = 0, Sigma^> = Sigma^< + Sigma^r - Sigma^r+ on
// every contact; which = 1, Sigma^r - Sigma^r+ = -i Gamma on contact 1 and
// zero on contact 0 (the transmission).
void launch_form_source(const Ctx& c, double2* src0, double2* src1, int which, int nb, hipStream_t st);
// diag of the G^< fronts' rows in the caller's site order into out[nE][n]
void launch_epilogue_lesser(const Ctx& c, int nb, double2* out, hipStream_t st);
// T(E) = -Tr[(Sigma^r_0 - Sigma^r_0+) X_00] from the G^< fronts' contact-0 block
void launch_transmission(const Ctx& c, const int32_t* caddr, int nb, double* T, hipStream_t st);

// Vector kernels of the Schroedinger-Poisson Newton step (kernels_poisson.hip):
// y = K x for a CSR matrix, out = a x + b y, *out = x . y (part: kVecBlocks
// doubles of scratch; fixed reduction order)
constexpr int kVecBlocks = 1024;
void launch_spmv(int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, const double* val,
                 const double* x, double* y, hipStream_t st);
void launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* out, hipStream_t st);
void launch_dot(int64_t n, const double* x, const double* y, double* part, double* out, hipStream_t st);
void launch_scba_mix(const double2* dgr, const double2* dgl, double2* sr, double2* sl, int64_t count,
                     double d0, double mix, double* part, double* out, hipStream_t st);

// Launchers (kernels.hip).  nb = energies in the batch.
void launch_assemble(const Ctx& c, const int32_t* cls, int ncl, int nb, hipStream_t st);
// cls_size: the largest cluster size s of the launch (selects the tile shape)
void launch_factor(const Ctx& c, const int32_t* cls, int ncl, int nb, int cls_size, hipStream_t st);
void launch_psi(const Ctx& c, const ColItem* it, int nit, int nb, int cls_size, hipStream_t st);
// tile_rows: 64, or 32 for clusters with s <= kUpdNarrowS (items of that height)
constexpr int kUpdNarrowS = 16;
void launch_update(const Ctx& c, const UpdItem* it, int nit, int nb, int tile_rows, hipStream_t st);
void launch_chain_fwd(const Ctx& c, const ChainItem* it, int nit, int nb, hipStream_t st);
void launch_down_off(const Ctx& c, const ColItem* it, int nit, int nb, bool lesser, int cls_size,
                     hipStream_t st);
void launch_down_diag(const Ctx& c, const int32_t* cls, int ncl, int nb, bool lesser, int cls_size,
                      hipStream_t st);
// T = Zd Sigma^< for all (chain cluster, contact) items at once (after the
// fold, before the back substitution, with the Ctx the latter will use)
void launch_chain_t(const Ctx& c, const ChainItem* it, int nit, int nb, hipStream_t st);
void launch_chain_back(const Ctx& c, const int32_t* cls, int ncl, int nb, hipStream_t st);
// small fronts: f <= 32 (one wave per front) or f <= 64 (four waves)
void launch_fold_small(const Ctx& c, const int32_t* cls, int ncl, int nb, int front_size, hipStream_t st);
// Small-front extraction: threads per block for a group's largest front, and
// how many (row pair, column) items of X_{i,B} a thread of such a block may
// hold in registers (ceil(s / 2) b is at most 136, 300, 528 for fronts of 32,
// 48, 64 points: two items cover all but the few 32-point leaves above 128).
constexpr int extract_threads(int front_size) { return front_size <= 32 ? 64 : front_size <= 48 ? 256 : 512; }
constexpr int extract_leaf_items(int) { return 2; }
void launch_extract_small(const Ctx& c, const int32_t* cls, int ncl, int nb, size_t lds_bytes, size_t lds_bytes_leaf,
                          int front_size, bool lesser, hipStream_t st);
constexpr int kSmallFront = 64;
constexpr int kMaxKids = 64;  // children per cluster (front assembly tables)  // fronts up to this size are handled whole on chip
void launch_fill_zero(double* p, int64_t count, hipStream_t st);
void launch_fill_zero_i32(int32_t* p, int64_t count, hipStream_t st);
void launch_advance(int32_t* e0, const int32_t* inc, int n, hipStream_t st);
// adjoint solves: clusters with s <= kRhsSmallS, b <= kRhsSmallB and
// s b <= kRhsSmallSB run one wavefront each (dynamic LDS rhs_small_lds_*),
// the others as 64 x 64 tiles (faster once the products grow)
constexpr int kRhsSmallS = 16, kRhsSmallB = 64, kRhsSmallSB = 512;
inline bool rhs_small_host(int s, int b) { return s <= kRhsSmallS && b <= kRhsSmallB && s * b <= kRhsSmallSB; }
inline size_t rhs_small_lds_fwd(int s, int b) { return (size_t)s * b * 16; }
inline size_t rhs_small_lds_back(int s, int b) { return (size_t)(s * b + s * s) * 16 + (size_t)b * 4; }
void launch_rhs_fwd(const Ctx& c, const RhsCtx& r, const int32_t* cls, int ncl, int nb, size_t small_lds,
                    bool big, hipStream_t st);
void launch_rhs_back(const Ctx& c, const RhsCtx& r, const int32_t* cls, int ncl, int nb, size_t small_lds,
                     bool big, hipStream_t st);
void launch_vjp_accum(const Ctx& c, const RhsCtx& r, int cc, int off, int nb, hipStream_t st);
void launch_zero(double* p, int64_t count, hipStream_t st);
void launch_vjp_reduce(const Ctx& c, const RhsCtx& r, int nb, const double* cE, double* vbar, hipStream_t st);
void launch_density(const Ctx& c, int nb, const double* cE, double* dens, hipStream_t st);
void launch_epilogue(const Ctx& c, int nb, double2* dgr, double2* dgl, double2* dgg, hipStream_t st);

}  // namespace ndg
