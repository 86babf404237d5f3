// HIP kernels for gfx950 (CDNA4): the fold (block LDL^T over the separator
// tree), the root inversion and the top-down extraction of G^r and G^<
// (Section 3.2), batched over energies x clusters of one tree level.
//
// Data: every (energy, cluster) owns dense complex128 blocks in HBM (see
// ClusterDesc).  Dense complex products run on the FP64 matrix cores:
// v_mfma_f64_16x16x4_f64 on split real/imaginary planes, four real MFMAs per
// complex 16x16x4 step, operands staged through LDS in 16-deep K chunks.
// Pivot blocks (s <= 64) are inverted on chip by Gauss-Jordan elimination
// with partial pivoting (row search by one wavefront's shuffles).
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace ndg {

// ---------------------------------------------------------------------------
// Fold: assemble the rows of cluster i of the front [i, B_i] of A^(l): its
// rows of A (entries towards i and B_i) plus the children's Schur
// contributions that land in those rows (extend-add).  Gathered: each entry
// sums its terms in registers and is written once, each child's term found
// through the child's map from this front's positions to its B indices
// (only the leading rows of a child's contribution, its parent's points,
// land in these rows).  The B x B block of the front is not formed: the
// Schur update gathers it from the children directly.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_assemble(Ctx c, const int32_t* cls) {
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  double2* F = S + d.o_fg;
  const int f = d.f, s = d.s;
  const int t = threadIdx.x;
  const double* hf = c.hfront + d.o_hf;
  const int32_t* smp = d.o_smap >= 0 ? c.smap + d.o_smap : nullptr;
  const double ez = c.E[eb + e];
  __shared__ int64_t kid_inv[kMaxKids], kid_upd[kMaxKids];
  __shared__ int kid_b[kMaxKids];
  const int k0 = c.kids_ptr[cl], nk = c.kids_ptr[cl + 1] - k0;
  for (int q = t; q < nk; q += 256) {
    const ClusterDesc& dc = c.cl[c.kids[k0 + q]];
    kid_inv[q] = dc.o_pinv;
    kid_upd[q] = dc.o_upd;
    kid_b[q] = dc.b;
  }
  __syncthreads();
  // -H, z - V on the diagonal, -Sigma, then the children's terms: one pass
  // over all s f entries, so short rows do not idle threads.  Four entries
  // per thread at a time, so that each round of dependent loads (map
  // entries, then the values they point to) is issued for all four at once;
  // the first child's map entries go out with the template's loads, and
  // each later child's before the previous child's values are waited for.
  const int nq = s * f;
  for (int q0 = t; q0 < nq; q0 += 4 * 256) {
    int ii[4], jj[4], qq[4];
    double re[4], im[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      qq[u] = min(q0 + u * 256, nq - 1);  // past the end: a repeat, not stored
      ii[u] = qq[u] / f;
      jj[u] = qq[u] - ii[u] * f;
      re[u] = hf[qq[u]];
      im[u] = 0.0;
    }
    int ri[4], rj[4];
    if (nk > 0) {
      const int32_t* inv = c.pinv + kid_inv[0];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ri[u] = inv[ii[u]];
        rj[u] = inv[jj[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (jj[u] == ii[u]) {
        const int site = c.perm[d.pt_off + ii[u]];
        re[u] += ez - (c.V ? c.V[site] : 0.0);
        im[u] = c.eta;
        if (c.sig_r_ph) {
          const double2 sp = c.sig_r_ph[(int64_t)(eb + e) * c.n + site];
          re[u] -= sp.x;
          im[u] -= sp.y;
        }
      }
    if (smp) {
      int code[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) code[u] = smp[qq[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (code[u] >= 0) {
          const int cc = code[u] >> 24, nc = sel2(c.nc, cc);
          const double2 sv = sel2(c.sig_r, cc)[(int64_t)(eb + e) * nc * nc + (code[u] & 0xFFFFFF)];
          re[u] -= sv.x;
          im[u] -= sv.y;
        }
    }
    for (int kq = 0; kq < nk; ++kq) {
      bool in[4];
      double2 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        in[u] = ri[u] >= 0 && rj[u] >= 0;
        // the contribution's upper triangle holds both (symmetric)
        if (in[u]) x[u] = S[kid_upd[kq] + (int64_t)min(ri[u], rj[u]) * kid_b[kq] + max(ri[u], rj[u])];
      }
      if (kq + 1 < nk) {
        const int32_t* inv = c.pinv + kid_inv[kq + 1];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ri[u] = inv[ii[u]];
          rj[u] = inv[jj[u]];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (in[u]) {
          re[u] += x[u].x;
          im[u] += x[u].y;
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q0 + u * 256 < nq) F[q0 + u * 256] = make_double2(re[u], im[u]);
  }
}

// ---------------------------------------------------------------------------
// Pivot block inverse by Gauss-Jordan elimination with partial pivoting, on
// chip (s <= 64).  Writes (A_ii^(fold))^{-1}; for the root this is G_root.
// ---------------------------------------------------------------------------
template <int SM, int NT>
__global__ void __launch_bounds__(NT) k_factor(Ctx c, const int32_t* cls) {
  // column groups of 16 (8 for the 16-point class): several columns per
  // thread, so the pivot row is published from a branch per register slot
  using GJ = RegGJ<SM, NT, (SM == 16 ? 8 : 16)>;
  static_assert(SM <= 64 || NT >= 512, "the 128-point inverse spreads over 512 threads");
  __shared__ typename GJ::Smem sm;
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  const double2* F = S + d.o_fg;
  const int f = d.f, s = d.s;
  const int t = threadIdx.x;
  GJ g(t);
#pragma unroll
  for (int m = 0; m < GJ::NR; ++m)
#pragma unroll
    for (int q = 0; q < GJ::NC; ++q) {
      const int i = g.row(m), j = g.col(q);
      const double2 v = (i < s && j < s) ? F[(int64_t)i * f + j] : cz();
      g.re[m][q] = v.x;
      g.im[m][q] = v.y;
    }
  const bool ok = g.run(sm, s);
  if (!ok && t == 0) raise_fault(c.status, -4, eb + e, cl);
  double2* Ainv = S + d.o_ainv;
#pragma unroll
  for (int m = 0; m < GJ::NR; ++m)
#pragma unroll
    for (int q = 0; q < GJ::NC; ++q) {
      const int i = g.row(m), j = g.col(q);
      if (i < s && j < s)
        Ainv[(int64_t)sm.pinv[i] * s + sm.piv[j]] = make_double2(g.re[m][q], g.im[m][q]);
    }
  if (c.growth && d.b > 0) {
    // ||A_ii^{-1}||_inf ||A_iB||_inf from the stored inverse, one row per lane
    __threadfence_block();
    __syncthreads();
    if (t < 64) {
      double ru = 0.0, rb = 0.0;
      for (int r = t; r < s; r += 64) {  // rows t, t + 64: fixed order per lane
        double u = 0.0, w = 0.0;
        for (int j = 0; j < s; ++j) {
          const double2 v = Ainv[(int64_t)r * s + j];
          u += sqrt(v.x * v.x + v.y * v.y);
        }
        const double2* row = F + (int64_t)r * f + s;
        for (int j = 0; j < d.b; ++j) w += sqrt(row[j].x * row[j].x + row[j].y * row[j].y);
        ru = fmax(ru, u);
        rb = fmax(rb, w);
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        ru = fmax(ru, __shfl_xor(ru, off));
        rb = fmax(rb, __shfl_xor(rb, off));
      }
      // non-negative doubles order like their bit patterns
      if (t == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(c.growth + eb + e),
                  (unsigned long long)__double_as_longlong(ru * rb));
    }
  }
}

// Psi_{i,B_i} = -A_ii^{-1} A_{i,B_i}: one 64-column tile per block.
template <int TM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 64 ? 2 : 3))) k_psi(Ctx c, const ColItem* items) {
  __shared__ GemmSmemR<TM> sm;
  const WorkIdx wk = xcd_work();
  const ColItem it = items[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[it.cl];
  double2* S = slab(c, e);
  const double2* Ainv = S + d.o_ainv;
  const double2* F = S + d.o_fg;
  double2* Psi = S + d.o_psi;
  const int s = d.s, b = d.b, f = d.f, j0 = it.tc * 64;
  const int nj = min(64, b - j0);
  // clusters of more than TM points (up to 128) take the rows in TM-row tiles
  for (int r0 = 0; r0 < s; r0 += TM) {
    const int ni = min(TM, s - r0);
    ZTile acc;
    ztile_zero(acc);
    zgemm_acc_t<TM, false, false>(
        s, [&](int i, int k) { return i < ni ? Ainv[(r0 + i) * s + k] : cz(); },
        [&](int k, int j) { return j < nj ? F[(int64_t)k * f + s + j0 + j] : cz(); }, acc, sm, ni, nj);
    ztile_store_t<TM>(acc, [&](int i, int j, double re, double im) {
      if (i < ni && j < nj) Psi[(int64_t)(r0 + i) * b + j0 + j] = make_double2(-re, -im);
    });
    __syncthreads();
  }
}

// Schur contribution of cluster i to its parent front:
// U = F_BB + Psi^T F_{i,B} (b x b), one TM x 64 tile per block.  Clusters
// with s <= 16 (K = s: the tile is all gather and store) take 32-row tiles:
// half the accumulators, more blocks in flight, less padding on ragged edges.
// U is complex symmetric (A is), so only its upper triangle is formed and
// stored (tiles wholly below the diagonal are not launched) and every
// reader takes entry (u, v) from (min(u, v), max(u, v)): half the bytes
// written, and one value for both triangles.
template <int TM, bool P64>
__device__ __forceinline__ void update_body(const Ctx& c, const UpdItem* items) {
  using GM = Gemm<P64>;
  __shared__ typename GM::template SmemT<TM> sm;
  const WorkIdx wk = xcd_work();
  const UpdItem it = items[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[it.cl];
  double2* S = slab(c, e);
  const double2* F = S + d.o_fg;
  const double2* Psi = S + d.o_psi;
  double2* U = S + d.o_upd;
  const int s = d.s, b = d.b, f = d.f;
  const int i0 = it.tr * TM, j0 = it.tc * 64;
  const int ni = min(TM, b - i0), nj = min(64, b - j0);
  // the children's index maps and contribution blocks (F_BB is gathered)
  __shared__ int64_t kid_inv[kMaxKids], kid_upd[kMaxKids];
  __shared__ int kid_b[kMaxKids];
  const int k0 = c.kids_ptr[it.cl], nk = c.kids_ptr[it.cl + 1] - k0;
  for (int q = threadIdx.x; q < nk; q += 256) {
    const ClusterDesc& dc = c.cl[c.kids[k0 + q]];
    kid_inv[q] = dc.o_pinv;
    kid_upd[q] = dc.o_upd;
    kid_b[q] = dc.b;
  }
  typename GM::Tile acc;
  GM::zero(acc);
  GM::template acc<TM, true, false, (TM != 64)>(
      s, [&](int i, int k) { return i < ni ? Psi[(int64_t)k * b + i0 + i] : cz(); },
      [&](int k, int j) { return j < nj ? F[(int64_t)k * f + s + j0 + j] : cz(); }, acc, sm, ni, nj);
  // F_BB gathered from the children: each lane holds fixed tile rows and
  // columns (lane l, register r -> column l%16 of each 16 x 16 block and row
  // l/16 + 4r for the FP64 matrix-core layout, 4(l/16) + r for the FP32
  // one), so their map entries are loaded once per child.  FP64 tiles take
  // the sum straight into the accumulators; with FP32 tiles it is kept in
  // FP64 and added when the tile is stored
  using T = TileShape<TM>;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
  double cr[T::MB][T::NB][4], ci[T::MB][T::NB][4];
#pragma unroll
  for (int m = 0; m < T::MB; ++m)
#pragma unroll
    for (int n = 0; n < T::NB; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) cr[m][n][r] = ci[m][n][r] = 0.0;
  for (int q = 0; q < nk; ++q) {
    const int32_t* inv = c.pinv + kid_inv[q];
    const double2* Uq = S + kid_upd[q];
    const int bq = kid_b[q];
    int cj[T::NB], ri[T::MB][4];
#pragma unroll
    for (int n = 0; n < T::NB; ++n) {
      const int j = wc + n * 16 + (lane & 15);
      cj[n] = j < nj ? inv[s + j0 + j] : -1;
    }
#pragma unroll
    for (int m = 0; m < T::MB; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr + m * 16 + (P64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        ri[m][r] = i < ni ? inv[s + i0 + i] : -1;
      }
#pragma unroll
    for (int m = 0; m < T::MB; ++m)
#pragma unroll
      for (int n = 0; n < T::NB; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (ri[m][r] >= 0 && cj[n] >= 0) {
            const int lo = min(ri[m][r], cj[n]), hi = max(ri[m][r], cj[n]);
            const double2 u = Uq[(int64_t)lo * bq + hi];
            if constexpr (P64) {
              acc.re[m][n][r] += u.x;
              acc.im[m][n][r] += u.y;
            } else {
              cr[m][n][r] += u.x;
              ci[m][n][r] += u.y;
            }
          }
  }
#pragma unroll
  for (int m = 0; m < T::MB; ++m)
#pragma unroll
    for (int n = 0; n < T::NB; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr + m * 16 + (P64 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        const int j = wc + n * 16 + (lane & 15);
        if (i < ni && j < nj && i0 + i <= j0 + j)
          U[(int64_t)(i0 + i) * b + j0 + j] =
              make_double2(cr[m][n][r] + (double)acc.re[m][n][r], ci[m][n][r] + (double)acc.im[m][n][r]);
      }
}

template <bool P64>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P64 ? 4 : 3)))
k_update(Ctx c, const UpdItem* items) {
  update_body<64, P64>(c, items);
}
template <bool P64>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_update_narrow(Ctx c, const UpdItem* items) {
  update_body<32, P64>(c, items);
}

// ---------------------------------------------------------------------------
// G^< source along a contact's chain (contact cluster and its ancestors).
// Forward solve L Z = E_c restricted to the chain: Z_c = I on the contact
// sites, Z_i = sum over chain descendants d coupled to i of Psi_{d,i}^T Z_d
// (passed up as V_d = Psi_d^T Z_d over B_d), then Zd_i = A_ii^{-1} Z_i.
// Zf rows [0, s) end up holding Zd_i, rows [s, f) the contribution V_i.
// ---------------------------------------------------------------------------
// fronts and contacts up to this many points keep the chain solve's index
// maps in LDS (larger ones read them from memory)
constexpr int kChainMap = 512;

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_chain_fwd(Ctx c, const ChainItem* items) {
  __shared__ GemmSmem sm;
  const WorkIdx wk = xcd_work();
  const ChainItem it = items[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[it.cl];
  const int cc = it.c, sc = sel2(c.nc, cc);
  double2* S = slab(c, e);
  double2* Zf = S + sel2(d.o_zf, cc);
  const double2* Psi = S + d.o_psi;
  const double2* Ainv = S + d.o_ainv;
  const int s = d.s, b = d.b, f = d.f;
  const int t = threadIdx.x;
  // The right-hand side over the front before the solve, read where it
  // lives: a one at each of the contact's sites held by this cluster (its
  // own column), else the chain child's contribution V_d at the positions
  // its B maps to, else zero.  Every entry of Zf is then written once.
  const int ch = sel2(d.chain_child, cc);
  const double2* Zc = nullptr;
  const int32_t* inv = nullptr;  // front position -> the child's B index, or -1
  int cs = 0;
  if (ch >= 0) {
    const ClusterDesc dc = c.cl[ch];
    Zc = S + sel2(dc.o_zf, cc);
    inv = c.pinv + dc.o_pinv;
    cs = dc.s;
  }
  const int32_t* pos = sel2(c.cpos, cc);
  const int off = d.pt_off;
  // the two maps in LDS, so that an entry of the right-hand side costs one
  // dependent global load instead of three
  __shared__ int rmap[kChainMap], cmap[kChainMap];
  const bool lmap = f <= kChainMap && sc <= kChainMap;
  if (lmap) {
    for (int p = t; p < f; p += 256) rmap[p] = inv ? inv[p] : -1;
    for (int a = t; a < sc; a += 256) cmap[a] = pos[a] - off;
  }
  __syncthreads();
  auto rhs = [&](int p, int a) {
    if (p < s && (lmap ? cmap[a] : pos[a] - off) == p) return make_double2(1.0, 0.0);
    const int r = lmap ? rmap[p] : (inv ? inv[p] : -1);
    return r >= 0 ? Zc[(int64_t)(cs + r) * sc + a] : cz();
  };
  // contacts wider than one tile: 64-column panels of Zf, independent
  for (int j0 = 0; j0 < sc; j0 += 64) {
    const int nj = min(64, sc - j0);
    // rows [s, f): V_i = rhs + Psi^T rhs_i
    for (int i0 = 0; i0 < b; i0 += 64) {
      const int ni = min(64, b - i0);
      ZTile acc;
      ztile_zero(acc);
      zgemm_acc<true, false>(
          s, [&](int i, int k) { return i < ni ? Psi[(int64_t)k * b + i0 + i] : cz(); },
          [&](int k, int j) { return j < nj ? rhs(k, j0 + j) : cz(); }, acc, sm, ni, nj);
      ztile_store_add_t<64, true>(
          acc, [&](int i, int j) { return (i < ni && j < nj) ? rhs(s + i0 + i, j0 + j) : cz(); },
          [&](int i, int j, double re, double im) {
            if (i < ni && j < nj) Zf[(int64_t)(s + i0 + i) * sc + j0 + j] = make_double2(re, im);
          });
    }
    // rows [0, s): Zd_i = A_ii^{-1} rhs_i, in 64-row tiles
    for (int r0 = 0; r0 < s; r0 += 64) {
      const int ni = min(64, s - r0);
      ZTile acc;
      ztile_zero(acc);
      zgemm_acc<false, false>(
          s, [&](int i, int k) { return i < ni ? Ainv[(r0 + i) * s + k] : cz(); },
          [&](int k, int j) { return j < nj ? rhs(k, j0 + j) : cz(); }, acc, sm, ni, nj);
      ztile_store(acc, [&](int i, int j, double re, double im) {
        if (i < ni && j < nj) Zf[(int64_t)(r0 + i) * sc + j0 + j] = make_double2(re, im);
      });
    }
  }
}

// T_i = Zd_i Sigma^<_c (s x sc) for every (chain cluster, contact): it needs
// only the forward solve's Zd_i and the source, so all chain clusters form
// it in one launch after the fold instead of inside the sequential back
// substitution.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_chain_t(Ctx c, const ChainItem* items) {
  __shared__ GemmSmem sm;
  const WorkIdx wk = xcd_work();
  const ChainItem it = items[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[it.cl];
  const int cc = it.c, sc = sel2(c.nc, cc), s = d.s;
  double2* S = slab(c, e);
  const double2* Zf = S + sel2(d.o_zf, cc);
  double2* T = S + sel2(d.o_t, cc);
  const double2* sl = sel2(c.sig_l, cc) + (int64_t)(eb + e - c.sl_e0) * sc * sc;
  for (int r0 = 0; r0 < s; r0 += 64)
    for (int j0 = 0; j0 < sc; j0 += 64) {
      const int ni = min(64, s - r0), nj = min(64, sc - j0);
      ZTile acc;
      ztile_zero(acc);
      zgemm_acc<false, false>(
          sc, [&](int i, int k) { return i < ni ? Zf[(int64_t)(r0 + i) * sc + k] : cz(); },
          [&](int k, int j) { return j < nj ? sl[(int64_t)k * sc + j0 + j] : cz(); }, acc, sm, ni, nj);
      ztile_store(acc, [&](int i, int j, double re, double im) {
        if (i < ni && j < nj) T[(int64_t)(r0 + i) * sc + j0 + j] = make_double2(re, im);
      });
    }
}

// Back substitution along the chain: X = rows of the contact's column of G^r,
// X_B gathered from the parent's front, X_i = Zd_i + Psi_i X_B.  Then the
// source of the G^< extraction on the cluster's rows:
// P_init = sum_c T_i (X_front)^+ (s x f) with T_i = Zd_i Sigma^<_c from
// k_chain_t, written into rows [0, s) of the G^< front.  This is
// D^{-1} L^{-1} Sigma^< (G^r)^+ restricted to the front, evaluated as
// (L^{-1} Sigma^<)(G^r)^+ so only s x sc panels are folded.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_chain_back(Ctx c, const int32_t* cls) {
  __shared__ GemmSmem sm;
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  double2* FP = S + d.o_fp;
  const int s = d.s, b = d.b, f = d.f;
  const int t = threadIdx.x;
  bool first = true;
  for (int cc = 0; cc < c.ncontacts; ++cc) {
    if (!((d.chain_mask >> cc) & 1)) continue;
    const int sc = sel2(c.nc, cc);
    double2* Xf = S + sel2(d.o_xf, cc);
    const double2* Zf = S + sel2(d.o_zf, cc);
    double2* T = S + sel2(d.o_t, cc);
    if (d.parent >= 0) {
      const ClusterDesc dp = c.cl[d.parent];
      const double2* Xp = S + sel2(dp.o_xf, cc);
      const int32_t* rel = c.relmap + d.bptr;
      for (int q = t; q < b * sc; q += 256) {
        const int r = q / sc, a = q % sc;
        Xf[(int64_t)(s + r) * sc + a] = Xp[(int64_t)rel[r] * sc + a];
      }
    }
    __syncthreads();
    // 64-row tiles of the cluster's rows (one unless s > 64)
    for (int r0 = 0; r0 < s; r0 += 64)
      for (int j0 = 0; j0 < sc; j0 += 64) {
        const int ni = min(64, s - r0), nj = min(64, sc - j0);
        ZTile acc;
        ztile_zero(acc);
        zgemm_acc_t<64, false, false, false>(
            b, [&](int i, int k) { return i < ni ? Psi[(int64_t)(r0 + i) * b + k] : cz(); },
            [&](int k, int j) { return j < nj ? Xf[(int64_t)(s + k) * sc + j0 + j] : cz(); }, acc, sm, ni, nj);
        ztile_store_add_t<64>(
            acc, [&](int i, int j) { return (i < ni && j < nj) ? Zf[(int64_t)(r0 + i) * sc + j0 + j] : cz(); },
            [&](int i, int j, double re, double im) {
              if (i < ni && j < nj) Xf[(int64_t)(r0 + i) * sc + j0 + j] = make_double2(re, im);
            });
      }
    __syncthreads();
    for (int r0 = 0; r0 < s; r0 += 64)
      for (int j0 = 0; j0 < f; j0 += 64) {
        const int ni = min(64, s - r0), nj = min(64, f - j0);
        ZTile acc;
        ztile_zero(acc);
        zgemm_acc_t<64, false, true, true>(
            sc, [&](int i, int k) { return i < ni ? T[(int64_t)(r0 + i) * sc + k] : cz(); },
            [&](int k, int j) {
              if (j >= nj) return cz();
              const double2 x = Xf[(int64_t)(j0 + j) * sc + k];
              return make_double2(x.x, -x.y);
            },
            acc, sm, ni, nj);
        ztile_store_add_t<64>(
            acc, [&](int i, int j) { return (!first && i < ni && j < nj) ? FP[(int64_t)(r0 + i) * f + j0 + j] : cz(); },
            [&](int i, int j, double re, double im) {
              if (i < ni && j < nj) FP[(int64_t)(r0 + i) * f + j0 + j] = make_double2(re, im);
            });
      }
    __syncthreads();
    first = false;
  }
}

// ---------------------------------------------------------------------------
// Extraction (top-down).  For cluster i:
//   G_{i,B} = Psi_i G_{B,B},        P_{i,B} = P_init + Psi_i P_{B,B},
// one 64-column tile per block.  G_{B,B} (P_{B,B}) is gathered from the
// stored rows of the clusters owning B (gather_bb): every cluster keeps only
// its own rows [G_ii, G_{i,B}], which its descendants read.
// ---------------------------------------------------------------------------
template <int TM, bool P64, int L>
__device__ __forceinline__ void down_off_body(const Ctx& c, const ColItem* items) {
  constexpr bool lesser = L != 0;
  using GM = Gemm<P64>;
  __shared__ typename GM::template SmemT<TM> sm;
  const WorkIdx wk = xcd_work();
  const ColItem it = items[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[it.cl];
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  double2* X = S + (lesser ? d.o_fp : d.o_fg);
  const int s = d.s, b = d.b, f = d.f, j0 = it.tc * 64;
  const int nj = min(64, b - j0);
  const bool has_src = lesser && (d.chain_mask || c.scat);
  const bool ls = lesser != 0;
  for (int r0 = 0; r0 < s; r0 += TM) {  // TM-row tiles (one unless s > TM)
    const int ni = min(TM, s - r0);
    typename GM::Tile acc;
    GM::zero(acc);
    auto fa = [&](int i, int k) { return i < ni ? Psi[(int64_t)(r0 + i) * b + k] : cz(); };
    if (d.o_bbd >= 0)
      GM::template acc<TM, false, false>(
          b, fa, [&](int k, int j) { return j < nj ? direct_bb(c, S, d, k, j0 + j, ls) : cz(); }, acc, sm, ni, nj);
    else if constexpr (P64)
      zgemm_acc_gather_t<TM, false>(
          b, fa, [&](int k, int j) { return j < nj ? gather_bb_entry(c, d, k, j0 + j) : 0; },
          [&](int32_t m, int j) { return j < nj ? gather_bb_value(c, S, m, ls) : cz(); }, acc, sm, ni, nj);
    else
      GM::template acc<TM, false, false>(
          b, fa, [&](int k, int j) { return j < nj ? gather_bb(c, S, d, k, j0 + j, ls) : cz(); }, acc, sm, ni, nj);
    if constexpr (P64) {
      ztile_store_add_t<TM>(
          acc, [&](int i, int j) { return (has_src && i < ni && j < nj) ? X[(int64_t)(r0 + i) * f + s + j0 + j] : cz(); },
          [&](int i, int j, double re, double im) {
            if (i < ni && j < nj) X[(int64_t)(r0 + i) * f + s + j0 + j] = make_double2(re, im);
          });
    } else {
      GM::template store<TM>(acc, [&](int i, int j, double re, double im) {
        if (i < ni && j < nj) {
          double2 v = make_double2(re, im);
          const int64_t pos = (int64_t)(r0 + i) * f + s + j0 + j;
          if (has_src) { const double2 p0 = X[pos]; v.x += p0.x; v.y += p0.y; }
          X[pos] = v;
        }
      });
    }
    if (r0 + TM < s) __syncthreads();
  }
}

// Occupancy targets without register spills (spilled registers go through
// scratch memory, costing HBM traffic): 64-row tiles two waves per SIMD,
// 32-row tiles three, 16-row tiles (bound by the gather of X_{B,B}, not the
// matrix cores) four.
template <int TM, bool P64, int L>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 64 ? 2 : 3)))
k_down_off(Ctx c, const ColItem* items) {
  down_off_body<TM, P64, L>(c, items);
}
template <bool P64, int L>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_down_off_narrow(Ctx c, const ColItem* items) {
  down_off_body<16, P64, L>(c, items);
}

//   G_ii = A_ii^{-1} + Psi_i G_{B,i},  G_{B,i} = G_{i,B}^T
//   P_ii = P_init + Psi_i P_{B,i},     P_{B,i} = -P_{i,B}^+
// Tile (r0, c0) of the block (TM x 64) as the product Psi_i X_{B,i} in acc.
template <int TM, bool P64, int L, bool PF = true, class SM>
__device__ __forceinline__ void down_diag_tile(const double2* Psi, const double2* X, int s, int b, int f, int r0,
                                               int c0, typename Gemm<P64>::Tile& acc, SM& sm) {
  using GM = Gemm<P64>;
  const int ni = min(TM, s - r0), nj = min(64, s - c0);
  GM::zero(acc);
  if constexpr (L != 0) {
    GM::template acc<TM, false, true, PF>(
        b, [&](int i, int k) { return i < ni ? Psi[(int64_t)(r0 + i) * b + k] : cz(); },
        [&](int k, int j) {
          if (j >= nj) return cz();
          const double2 x = X[(int64_t)(c0 + j) * f + s + k];
          return make_double2(-x.x, x.y);
        },
        acc, sm, ni, nj);
  } else {
    GM::template acc<TM, false, true, PF>(
        b, [&](int i, int k) { return i < ni ? Psi[(int64_t)(r0 + i) * b + k] : cz(); },
        [&](int k, int j) { return j < nj ? X[(int64_t)(c0 + j) * f + s + k] : cz(); }, acc, sm, ni, nj);
  }
}

// Blocks larger than one tile (and the FP32 tiles of the mixed path): TM x
// 64 tiles, each stored with U_i (G) or the source (P) added, then the
// block replaced by its symmetric (G) or anti-Hermitian (P) part in place.
template <int TM, bool P64, int L>
__device__ __forceinline__ void down_diag_body(const Ctx& c, const int32_t* cls) {
  constexpr bool lesser = L != 0;
  using GM = Gemm<P64>;
  __shared__ typename GM::template SmemT<TM> sm;
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  const double2* Ainv = S + d.o_ainv;
  double2* X = S + (lesser ? d.o_fp : d.o_fg);
  const int s = d.s, b = d.b, f = d.f;
  const bool has_src = lesser && (d.chain_mask || c.scat);
  // the block's columns [0, s) are written, its columns [s, f) only read
  for (int r0 = 0; r0 < s; r0 += TM)
    for (int c0 = 0; c0 < s; c0 += 64) {
      const int ni = min(TM, s - r0), nj = min(64, s - c0);
      typename GM::Tile acc;
      down_diag_tile<TM, P64, L>(Psi, X, s, b, f, r0, c0, acc, sm);
      GM::template store<TM>(acc, [&](int i, int j, double re, double im) {
        if (i < ni && j < nj) {
          double2 v = make_double2(re, im);
          const int64_t pos = (int64_t)(r0 + i) * f + c0 + j;
          if constexpr (lesser) {
            if (has_src) { const double2 p0 = X[pos]; v.x += p0.x; v.y += p0.y; }
          } else {
            const double2 a = Ainv[(r0 + i) * s + c0 + j];
            v.x += a.x;
            v.y += a.y;
          }
          X[pos] = v;
        }
      });
      if (r0 + TM < s || c0 + 64 < s) __syncthreads();
    }
  symmetrize_block(X, s, f, lesser);
}

// Blocks of one tile (s <= TM <= 64, FP64): the symmetric (G) or
// anti-Hermitian (P) part formed on chip, the transposed entries exchanged
// through the staging memory (free once the product is done) one plane at a
// time, and every entry written once.
template <int TM, int L>
__device__ __forceinline__ void down_diag_single_body(const Ctx& c, const int32_t* cls) {
  constexpr bool lesser = L != 0;
  __shared__ GemmSmemR<TM> sm;
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  const double2* Ainv = S + d.o_ainv;
  double2* X = S + (lesser ? d.o_fp : d.o_fg);
  const int s = d.s, b = d.b, f = d.f;
  const bool has_src = lesser && (d.chain_mask || c.scat);
  ZTile acc;
  down_diag_tile<TM, true, L, TM != 64>(Psi, X, s, b, f, 0, 0, acc, sm);
  // the block before symmetrization: the product plus U_i (G) or the
  // source (P, on the contact chains)
  ztile_apply_t<TM>(acc, [&](int i, int j, double& re, double& im) {
    if (i < s && j < s) {
      if constexpr (lesser) {
        if (has_src) {
          const double2 p0 = X[(int64_t)i * f + j];
          re += p0.x;
          im += p0.y;
        }
      } else {
        const double2 a = Ainv[i * s + j];
        re += a.x;
        im += a.y;
      }
    }
  });
  constexpr int LD = TM + 1;
  static_assert(sizeof(sm) >= sizeof(double) * TM * LD, "staging holds one plane");
  double* plane = reinterpret_cast<double*>(&sm);
  double* Xd = reinterpret_cast<double*>(X);
  for (int part = 0; part < 2; ++part) {
    __syncthreads();
    ztile_store_t<TM>(acc, [&](int i, int j, double re, double im) {
      if (i < s && j < s) plane[i * LD + j] = part ? im : re;
    });
    __syncthreads();
    ztile_store_t<TM>(acc, [&](int i, int j, double re, double im) {
      if (i < s && j < s) {
        const double t = plane[j * LD + i];
        // (X + X^T) / 2, or (X - X^+) / 2: real parts subtract
        const double o = part ? 0.5 * (im + t) : (lesser ? 0.5 * (re - t) : 0.5 * (re + t));
        Xd[2 * (i * f + j) + part] = o;
      }
    });
  }
}

// Entry points as for k_down_off (occupancy without spills).
template <int TM, bool P64, int L>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 64 ? 2 : 3)))
k_down_diag(Ctx c, const int32_t* cls) {
  down_diag_body<TM, P64, L>(c, cls);
}
template <bool P64, int L>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
k_down_diag_narrow(Ctx c, const int32_t* cls) {
  down_diag_body<16, P64, L>(c, cls);
}
template <int TM, int L>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 64 ? 4 : 3)))
k_down_diag_single(Ctx c, const int32_t* cls) {
  down_diag_single_body<TM, L>(c, cls);
}

// diag G^r, G^<, G^> in the caller's site order; G^> = G^< + G^r - (G^r)^*.
__global__ void __launch_bounds__(256) k_epilogue(Ctx c, double2* dgr, double2* dgl, double2* dgg) {
  const int q = blockIdx.x * 256 + threadIdx.x;  // site in the caller's order
  const int e = blockIdx.y;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  if (q >= c.n) return;
  const SiteDiag sd = c.sdiag[q];
  const double2* S = slab(c, e);
  const double2 gr = S[sd.og];
  const double2 gl = S[sd.ol];
  const int64_t o = (int64_t)(eb + e) * c.n + q;
  dgr[o] = gr;
  dgl[o] = gl;
  if (dgg) dgg[o] = make_double2(gl.x, gl.y + 2.0 * gr.y);
  if (!isfinite(gr.x) || !isfinite(gr.y) || !isfinite(gl.x) || !isfinite(gl.y))
    raise_fault(c.status, -7, eb + e, sd.cl);
}

// Graph replays over an energy range: each plan's first energy advances by
// its batch size.
__global__ void k_advance(int32_t* e0, const int32_t* inc, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) e0[i] += inc[i];
}

__global__ void k_fill_zero_i32(int32_t* p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0;
}

__global__ void k_fill_zero(double* p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
void launch_advance(int32_t* e0, const int32_t* inc, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_advance, dim3((n + 255) / 256), dim3(256), 0, st, e0, inc, n);
}
void launch_fill_zero_i32(int32_t* p, int64_t count, hipStream_t st) {
  if (count > 0)
    hipLaunchKernelGGL(k_fill_zero_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count);
}
void launch_fill_zero(double* p, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count);
}
void launch_assemble(const Ctx& c, const int32_t* cls, int ncl, int nb, hipStream_t st) {
  if (ncl > 0) hipLaunchKernelGGL(k_assemble, dim3(ncl, nb), dim3(256), 0, st, c, cls);
}
void launch_factor(const Ctx& c, const int32_t* cls, int ncl, int nb, int cls_size, hipStream_t st) {
  if (ncl <= 0) return;
  if (cls_size <= 16) hipLaunchKernelGGL((k_factor<16, 64>), dim3(ncl, nb), dim3(64), 0, st, c, cls);
  else if (cls_size <= 32) hipLaunchKernelGGL((k_factor<32, 128>), dim3(ncl, nb), dim3(128), 0, st, c, cls);
  else if (cls_size <= 64) hipLaunchKernelGGL((k_factor<64, 256>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
  else hipLaunchKernelGGL((k_factor<128, 512>), dim3(ncl, nb), dim3(512), 0, st, c, cls);
}
void launch_psi(const Ctx& c, const ColItem* it, int nit, int nb, int cls_size, hipStream_t st) {
  if (nit <= 0) return;
  if (cls_size <= 16) hipLaunchKernelGGL((k_psi<16>), dim3(nit, nb), dim3(256), 0, st, c, it);
  else if (cls_size <= 32) hipLaunchKernelGGL((k_psi<32>), dim3(nit, nb), dim3(256), 0, st, c, it);
  else hipLaunchKernelGGL((k_psi<64>), dim3(nit, nb), dim3(256), 0, st, c, it);
}
void launch_update(const Ctx& c, const UpdItem* it, int nit, int nb, int tile_rows, hipStream_t st) {
  if (nit <= 0) return;
  if (tile_rows == 32) {
    if (c.mixed) hipLaunchKernelGGL((k_update_narrow<false>), dim3(nit, nb), dim3(256), 0, st, c, it);
    else hipLaunchKernelGGL((k_update_narrow<true>), dim3(nit, nb), dim3(256), 0, st, c, it);
  } else {
    if (c.mixed) hipLaunchKernelGGL((k_update<false>), dim3(nit, nb), dim3(256), 0, st, c, it);
    else hipLaunchKernelGGL((k_update<true>), dim3(nit, nb), dim3(256), 0, st, c, it);
  }
}
void launch_chain_fwd(const Ctx& c, const ChainItem* it, int nit, int nb, hipStream_t st) {
  if (nit > 0) hipLaunchKernelGGL(k_chain_fwd, dim3(nit, nb), dim3(256), 0, st, c, it);
}
template <bool P64, int L>
static void down_off_t(const Ctx& c, const ColItem* it, int nit, int nb, int cls_size, hipStream_t st) {
  if (cls_size <= 16) hipLaunchKernelGGL((k_down_off_narrow<P64, L>), dim3(nit, nb), dim3(256), 0, st, c, it);
  else if (cls_size <= 32) hipLaunchKernelGGL((k_down_off<32, P64, L>), dim3(nit, nb), dim3(256), 0, st, c, it);
  else hipLaunchKernelGGL((k_down_off<64, P64, L>), dim3(nit, nb), dim3(256), 0, st, c, it);
}
void launch_down_off(const Ctx& c, const ColItem* it, int nit, int nb, bool lesser, int cls_size,
                     hipStream_t st) {
  if (nit <= 0) return;
  if (c.mixed) {
    if (lesser) down_off_t<false, 1>(c, it, nit, nb, cls_size, st);
    else down_off_t<false, 0>(c, it, nit, nb, cls_size, st);
  } else {
    if (lesser) down_off_t<true, 1>(c, it, nit, nb, cls_size, st);
    else down_off_t<true, 0>(c, it, nit, nb, cls_size, st);
  }
}
template <bool P64, int L>
static void down_diag_t(const Ctx& c, const int32_t* cls, int ncl, int nb, int cls_size, hipStream_t st) {
  if constexpr (P64) {
    // FP64 blocks of one tile (every cluster of the group has s <= cls_size),
    // larger blocks in 64-row tiles
    if (cls_size <= 16) hipLaunchKernelGGL((k_down_diag_single<16, L>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
    else if (cls_size <= 32) hipLaunchKernelGGL((k_down_diag_single<32, L>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
    else if (cls_size <= 64) hipLaunchKernelGGL((k_down_diag_single<64, L>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
    else hipLaunchKernelGGL((k_down_diag<64, true, L>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
  } else {
    if (cls_size <= 16) hipLaunchKernelGGL((k_down_diag_narrow<false, L>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
    else if (cls_size <= 32) hipLaunchKernelGGL((k_down_diag<32, false, L>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
    else hipLaunchKernelGGL((k_down_diag<64, false, L>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
  }
}
void launch_down_diag(const Ctx& c, const int32_t* cls, int ncl, int nb, bool lesser, int cls_size,
                      hipStream_t st) {
  if (ncl <= 0) return;
  if (c.mixed) {
    if (lesser) down_diag_t<false, 1>(c, cls, ncl, nb, cls_size, st);
    else down_diag_t<false, 0>(c, cls, ncl, nb, cls_size, st);
  } else {
    if (lesser) down_diag_t<true, 1>(c, cls, ncl, nb, cls_size, st);
    else down_diag_t<true, 0>(c, cls, ncl, nb, cls_size, st);
  }
}
void launch_chain_t(const Ctx& c, const ChainItem* it, int nit, int nb, hipStream_t st) {
  if (nit > 0) hipLaunchKernelGGL(k_chain_t, dim3(nit, nb), dim3(256), 0, st, c, it);
}
void launch_chain_back(const Ctx& c, const int32_t* cls, int ncl, int nb, hipStream_t st) {
  if (ncl > 0) hipLaunchKernelGGL(k_chain_back, dim3(ncl, nb), dim3(256), 0, st, c, cls);
}
void launch_epilogue(const Ctx& c, int nb, double2* dgr, double2* dgl, double2* dgg, hipStream_t st) {
  hipLaunchKernelGGL(k_epilogue, dim3((c.n + 255) / 256, nb), dim3(256), 0, st, c, dgr, dgl, dgg);
}

}  // namespace ndg
