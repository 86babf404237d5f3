// Small fronts (f = s + b <= 64) handled whole on chip, one block per
// (energy, cluster).  Most clusters of a nested-dissection tree are small
// (leaves and the separators just above them), and tiling their products
// into 64 x 64 matrix-core tiles would mostly multiply padding.
//
// Fold: the front [[F_ii, F_iB], [F_Bi, F_BB]] is assembled directly in
// registers (the cluster's rows of A from a precomputed -H template, the
// children's contributions gathered through their index maps) and reduced by
// s steps of Gauss-Jordan elimination with partial pivoting among the rows of
// cluster i, applied to the whole front.  The result is
//     [[ F_ii^{-1},          F_ii^{-1} F_iB           ],
//      [ -F_Bi F_ii^{-1},    F_BB - F_Bi F_ii^{-1} F_iB ]]
// i.e. the pivot inverse, -Psi_{i,B}, Psi^T and the Schur contribution to the
// parent front (Section 3.2, fold: Psi_ij = -A_ii^{-1} A_ij and
// A_jk += Psi_ij^T A_ik for j, k in B_i) -- all in one pass.
//
// Extraction: G_{i,B} = Psi G_{B,B}, G_ii = A_ii^{-1} + Psi G_{B,i}, and the
// same with P (G^<), with the gathered B x B blocks and Psi held in LDS.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace ndg {

template <int SF, int NT, int JS>
__device__ __forceinline__ void fold_small_body(const Ctx& c, const int32_t* cls) {
  using GJ = RegGJ<SF, NT, JS>;
  __shared__ typename GJ::Smem gsm;
  __shared__ double rsum[2][SF];  // growth indicator: row sums of |F_iB| and |F_ii^{-1}|
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  const int f = d.f, s = d.s, b = d.b;
  const int t = threadIdx.x;
  GJ g(t);
  // the cluster's rows of A = zI - H - V - Sigma over the front (B rows by
  // symmetry), straight into the register tiles
  const double* hf = c.hfront + d.o_hf;
  const double ez = c.E[eb + e];
#pragma unroll
  for (int m = 0; m < GJ::NR; ++m)
#pragma unroll
    for (int q = 0; q < GJ::NC; ++q) {
      const int i = g.row(m), j = g.col(q);
      double re = 0.0, im = 0.0;
      if (i < f && j < f) {
        if (i < s) re = hf[i * f + j];
        else if (j < s) re = hf[j * f + i];
        if (i == j && i < s) {
          const int site = c.perm[d.pt_off + i];
          re += ez - (c.V ? c.V[site] : 0.0);
          im += c.eta;
          if (c.sig_r_ph) {
            const double2 sp = c.sig_r_ph[(int64_t)(eb + e) * c.n + site];
            re -= sp.x;
            im -= sp.y;
          }
        }
      }
      g.re[m][q] = re;
      g.im[m][q] = im;
    }
  if (d.o_smap >= 0) {
    const int32_t* smp = c.smap + d.o_smap;
#pragma unroll
    for (int m = 0; m < GJ::NR; ++m)
#pragma unroll
      for (int q = 0; q < GJ::NC; ++q) {
        const int i = g.row(m), j = g.col(q);
        const int code = (i < f && j < f) ? smp[i * f + j] : -1;
        if (code >= 0) {
          const int cc = code >> 24, nc = sel2(c.nc, cc);
          const double2 sv = sel2(c.sig_r, cc)[(int64_t)(eb + e) * nc * nc + (code & 0xFFFFFF)];
          g.re[m][q] -= sv.x;
          g.im[m][q] -= sv.y;
        }
      }
  }
  // children's Schur contributions, gathered through their index maps
  for (int kp = c.kids_ptr[cl]; kp < c.kids_ptr[cl + 1]; ++kp) {
    const ClusterDesc dc = c.cl[c.kids[kp]];
    const int32_t* inv = c.pinv + dc.o_pinv;
    const double2* U = S + dc.o_upd;
    int ri[GJ::NR], cj[GJ::NC];
#pragma unroll
    for (int m = 0; m < GJ::NR; ++m) ri[m] = g.row(m) < f ? inv[g.row(m)] : -1;
#pragma unroll
    for (int q = 0; q < GJ::NC; ++q) cj[q] = g.col(q) < f ? inv[g.col(q)] : -1;
#pragma unroll
    for (int m = 0; m < GJ::NR; ++m)
#pragma unroll
      for (int q = 0; q < GJ::NC; ++q)
        if (ri[m] >= 0 && cj[q] >= 0) {
          // the contribution's upper triangle holds both (symmetric)
          const double2 u = U[min(ri[m], cj[q]) * dc.b + max(ri[m], cj[q])];
          g.re[m][q] += u.x;
          g.im[m][q] += u.y;
        }
  }
  // Row sums for the growth indicator: a row's JS owners are consecutive
  // lanes (thread t holds columns t % JS + JS q), so a butterfly over them
  // adds in a fixed order and the lane with jt = 0 stores the sum.
  auto row_sums = [&](double(&dst)[SF], bool inverse) {
#pragma unroll
    for (int m = 0; m < GJ::NR; ++m) {
      const int i = g.row(m);
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < GJ::NC; ++q) {
        const int j = g.col(q);
        if (i < s && (inverse ? j < s : (j >= s && j < f)))
          acc += sqrt(g.re[m][q] * g.re[m][q] + g.im[m][q] * g.im[m][q]);
      }
#pragma unroll
      for (int off = JS / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
      if (g.jt == 0 && i < s) dst[i] = acc;
    }
  };
  if (c.growth) row_sums(rsum[0], false);
  const bool ok = g.run(gsm, s);
  if (!ok && t == 0) raise_fault(c.status, -4, eb + e, cl);
  double2* Ainv = S + d.o_ainv;
  double2* Psi = S + d.o_psi;
  double2* Upd = S + d.o_upd;
  // storage row p_k holds row k of [A_ii^{-1}, A_ii^{-1} A_iB]; columns
  // below s are permuted the same way
#pragma unroll
  for (int m = 0; m < GJ::NR; ++m)
#pragma unroll
    for (int q = 0; q < GJ::NC; ++q) {
      const int i = g.row(m), j = g.col(q);
      const double vr = g.re[m][q], vi = g.im[m][q];
      if (i < s) {
        if (j < s) Ainv[gsm.pinv[i] * s + gsm.piv[j]] = make_double2(vr, vi);
        else if (j < f) Psi[gsm.pinv[i] * b + (j - s)] = make_double2(-vr, -vi);
      } else if (i < f && j >= i && j < f) {
        // the Schur contribution is complex symmetric: its upper triangle
        Upd[(i - s) * b + (j - s)] = make_double2(vr, vi);
      }
    }
  if (c.growth && b > 0) {
    // ||A_ii^{-1}||_inf ||A_iB||_inf (row sums are permutation invariant)
    row_sums(rsum[1], true);
    __syncthreads();
    if (t < 64) {
      double ru = 0.0, rb = 0.0;
      if (t < s) {
        ru = rsum[1][t];
        rb = rsum[0][t];
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        ru = fmax(ru, __shfl_xor(ru, off));
        rb = fmax(rb, __shfl_xor(rb, off));
      }
      if (t == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(c.growth + eb + e),
                  (unsigned long long)__double_as_longlong(ru * rb));
    }
  }
}

// Entry points: the 32-, 40- and 64-point classes fit 128 registers, so four
// wavefronts per SIMD; the 48-point class runs four wavefronts per front
// (three rows and three columns per thread) in 85 registers, five per SIMD;
// the 24-point class fits 102 (five), the most it takes without spills.
template <int SF, int NT, int JS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
k_fold_small(Ctx c, const int32_t* cls) {
  fold_small_body<SF, NT, JS>(c, cls);
}
template <int SF, int NT, int JS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(5)))
k_fold_small_narrow(Ctx c, const int32_t* cls) {
  fold_small_body<SF, NT, JS>(c, cls);
}

// Extraction of G^r (which = 0) or G^< (which = 1) for one small front; the
// two run as separate launches on two streams.  X_{B,B} is gathered from the
// stored rows of the clusters owning B (gather_bb).  Dynamic LDS holds
// Psi (s x b), the gathered upper triangle of the B x B block of the parent's
// front (the space later holds X_ii) and X_{i,B}.
// A leaf's blocks are read by nobody but the epilogue, so a leaf forms and
// stores only the diagonal of X_ii.
template <int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8)))
k_extract_small(Ctx c, const int32_t* cls, int which) {
  extern __shared__ double2 sm[];
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  const int f = d.f, s = d.s, b = d.b;
  const int lb = b | 1;           // odd row stride: lanes reading down a column hit distinct banks
  const int t = threadIdx.x;
  // with phonon sources every cluster's full rows [X_ii, X_{i,B}] are read
  // (by the all-ancestor extraction) and every cluster has a G^< source; a
  // contact's clusters keep full rows for the terminal currents
  const bool inner = c.scat || d.chain_mask != 0 || c.kids_ptr[cl + 1] > c.kids_ptr[cl];
  const bool chain = c.scat || d.chain_mask != 0;
  // a leaf forms only the diagonal of X_ii: its X_{i,B} can replace X_{B,B}
  // in LDS (the launch sizes LDS for that when no cluster is inner)
  constexpr int kLeafItems = extract_leaf_items(NT);
  const bool leaf = !inner && ((s + 1) >> 1) * b <= kLeafItems * NT;
  const double2* Ainv = S + d.o_ainv;
  double2* Psl = sm;              // s x b, stride lb
  double2* XBB = sm + s * lb;     // upper triangle of X_{B,B}, row-major
  const int ls = s | 1;           // odd row stride of X_ii (its transpose is read)
  const int ntri = b * (b + 1) / 2;
  // s x b, stride lb (X_{B,B} is later X_ii; a leaf's X_{i,B} replaces it)
  double2* XIB = leaf ? XBB : XBB + max(ntri, s * ls);
  double2* XII = XBB;
  const double2* Psi = S + d.o_psi;
  // two entries per thread at a time (their loads in flight together)
  for (int q0 = t; q0 < s * b; q0 += 2 * NT) {
    const int q1 = min(q0 + NT, s * b - 1);  // past the end: a repeat, not stored
    const double2 v0 = Psi[q0], v1 = Psi[q1];
    Psl[(q0 / b) * lb + q0 % b] = v0;
    if (q0 + NT < s * b) Psl[(q1 / b) * lb + q1 % b] = v1;
  }
  {
    const int lesser = which;
    double2* X = S + (lesser ? d.o_fp : d.o_fg);
    const bool src = lesser && chain;
    // X_{B,B} is complex symmetric for G^r and anti-Hermitian for G^<
    // (X_vu = -conj(X_uv)): only the upper triangle is gathered and kept.
    // Entry q of the triangle is (k, j), k <= j, rows of length b - k
    // starting at k b - k (k - 1) / 2.
    const float bh = (float)b + 0.5f;
    // four entries per thread at a time (their table entries, then their
    // values, loaded together) where the triangle spans several rounds of
    // the block; one at a time on tiny fronts
    if (ntri > 2 * NT) {
      for (int q0 = t; q0 < ntri; q0 += 4 * NT) {
        int jj[4];
        int32_t m[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + u * NT;
          int k = (int)(bh - sqrtf(bh * bh - 2.0f * (float)q));
          k = min(max(k, 0), b - 1);
          if (k * b - (k * (k - 1) >> 1) > q) --k;
          else if (k + 1 < b && (k + 1) * b - ((k + 1) * k >> 1) <= q) ++k;
          jj[u] = k + q - (k * b - (k * (k - 1) >> 1));
          if (q < ntri) m[u] = gather_bb_entry(c, d, k, jj[u]);
        }
        double2 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q0 + u * NT < ntri) x[u] = gather_bb_value(c, S, m[u], lesser != 0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q0 + u * NT < ntri) XBB[q0 + u * NT] = x[u];
      }
    } else {
      for (int q = t; q < ntri; q += NT) {
        int k = (int)(bh - sqrtf(bh * bh - 2.0f * (float)q));
        k = min(max(k, 0), b - 1);
        if (k * b - (k * (k - 1) >> 1) > q) --k;
        else if (k + 1 < b && (k + 1) * b - ((k + 1) * k >> 1) <= q) ++k;
        const int j = k + q - (k * b - (k * (k - 1) >> 1));
        XBB[q] = gather_bb(c, S, d, k, j, lesser != 0);
      }
    }
    __syncthreads();
    // X_{i,B} = P_init + Psi X_{B,B}: two rows per thread share each X_{B,B}
    // operand (rows r0 and r0 + 1, one column)
    const int sp2 = (s + 1) >> 1;
    // item q: rows r0 = 2 (q / b) and r0 + 1 (if any), column j = q % b
    auto item = [&](int q, double2& a0, double2& a1) {
      const int r0 = (q / b) << 1, j = q - (q / b) * b;
      const bool two = r0 + 1 < s;
      a0 = src ? X[(int64_t)r0 * f + s + j] : cz();
      a1 = (src && two) ? X[(int64_t)(r0 + 1) * f + s + j] : cz();
      const double2* p0r = Psl + r0 * lb;
      const double2* p1r = Psl + (two ? r0 + 1 : r0) * lb;
      // X_{B,B}[k][j]: (k, j) of the triangle for k <= j, at up (from (0, j)
      // = j, each row b - k - 1 further on), else the mirror of (j, k), at
      // mj + k
      const int mj = j * b - ((j * (j - 1)) >> 1) - j;
      int up = j;
      for (int k = 0; k < b; ++k) {
        const bool upper = k <= j;
        double2 x = XBB[upper ? up : mj + k];
        if (lesser && !upper) x.x = -x.x;
        up += upper ? b - k - 1 : 0;
        const double2 p0 = p0r[k], p1 = p1r[k];
        cmac(a0, p0, x);
        cmac(a1, p1, x);
      }
    };
    auto put = [&](int q, const double2& a0, const double2& a1) {
      const int r0 = (q / b) << 1, j = q - (q / b) * b;
      XIB[r0 * lb + j] = a0;
      if (r0 + 1 < s) XIB[(r0 + 1) * lb + j] = a1;
    };
    if (leaf) {
      // X_{i,B} takes the space of X_{B,B} once every thread has read that,
      // so it waits in registers (at most kLeafItems items per thread; a
      // leaf with more keeps X_{i,B} apart, as an inner cluster does)
      double2 v0[kLeafItems], v1[kLeafItems];
#pragma unroll
      for (int it = 0; it < kLeafItems; ++it)
        if (t + it * NT < sp2 * b) item(t + it * NT, v0[it], v1[it]);
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kLeafItems; ++it)
        if (t + it * NT < sp2 * b) put(t + it * NT, v0[it], v1[it]);
    } else {
      for (int q = t; q < sp2 * b; q += NT) {
        double2 a0, a1;
        item(q, a0, a1);
        put(q, a0, a1);
      }
    }
    __syncthreads();
    // X_ii = (A_ii^{-1} | P_init) + Psi X_{B,i};  X_{B,i}[k][j] = X_{i,B}[j][k]
    // for G^r, -conj(X_{i,B}[j][k]) for G^<.  A leaf's blocks are read by
    // nobody but the epilogue: it forms the diagonal only.
    const double sg = lesser ? -1.0 : 1.0;
    if (!inner) {
      for (int r = t; r < s; r += NT) {
        double2 a0 = lesser ? (src ? X[(int64_t)r * f + r] : cz()) : Ainv[r * s + r], a1 = cz();
        const double2* pr = Psl + r * lb;
        const double2* xr = XIB + r * lb;
        int k = 0;
        for (; k + 1 < b; k += 2) {
          const double2 p0 = pr[k], p1 = pr[k + 1];
          cmac(a0, p0, make_double2(sg * xr[k].x, xr[k].y));
          cmac(a1, p1, make_double2(sg * xr[k + 1].x, xr[k + 1].y));
        }
        if (k < b) cmac(a0, pr[k], make_double2(sg * xr[k].x, xr[k].y));
        X[(int64_t)r * f + r] = make_double2(a0.x + a1.x, a0.y + a1.y);
      }
    } else {
      // two rows per thread share each X_{B,i} operand; X_ii goes to the
      // LDS of X_{B,B} (no longer read; sized for s x s too) and its
      // symmetric (G) or anti-Hermitian (P) part to HBM once
      for (int q = t; q < sp2 * s; q += NT) {
        const int r0 = (q / s) << 1, j = q - (q / s) * s;
        const bool two = r0 + 1 < s;
        const int r1 = two ? r0 + 1 : r0;
        double2 a0 = lesser ? (src ? X[(int64_t)r0 * f + j] : cz()) : Ainv[r0 * s + j];
        double2 a1 = lesser ? (src ? X[(int64_t)r1 * f + j] : cz()) : Ainv[r1 * s + j];
        const double2* p0r = Psl + r0 * lb;
        const double2* p1r = Psl + r1 * lb;
        const double2* xr = XIB + j * lb;
        for (int k = 0; k < b; ++k) {
          const double2 x = make_double2(sg * xr[k].x, xr[k].y);
          cmac(a0, p0r[k], x);
          cmac(a1, p1r[k], x);
        }
        XII[r0 * ls + j] = a0;
        if (two) XII[r1 * ls + j] = a1;
      }
    }
    if (inner) {
      // the cluster's rows [X_ii, X_{i,B}] are what its descendants gather:
      // X_ii as (X + X^T) / 2 for G^r, (X - X^+) / 2 for G^< (one value
      // for both triangles, whichever a descendant reads)
      __syncthreads();
      for (int q = t; q < s * s; q += NT) {
        const int r = q / s, j = q - r * s;
        const double2 a = XII[r * ls + j], bt = XII[j * ls + r];
        X[(int64_t)r * f + j] = lesser ? make_double2(0.5 * (a.x - bt.x), 0.5 * (a.y + bt.y))
                                       : make_double2(0.5 * (a.x + bt.x), 0.5 * (a.y + bt.y));
      }
      for (int q = t; q < s * b; q += NT) {
        const int r = q / b, j = q - r * b;
        X[(int64_t)r * f + s + j] = XIB[r * lb + j];
      }
    }
    __syncthreads();
  }
}

void launch_fold_small(const Ctx& c, const int32_t* cls, int ncl, int nb, int front_size, hipStream_t st) {
  if (ncl <= 0) return;
  // the variant follows the largest front of the group (padding costs work
  // in every elimination step)
  if (front_size <= 24) hipLaunchKernelGGL((k_fold_small_narrow<24, 64, 8>), dim3(ncl, nb), dim3(64), 0, st, c, cls);
  else if (front_size <= 32) hipLaunchKernelGGL((k_fold_small<32, 64, 8>), dim3(ncl, nb), dim3(64), 0, st, c, cls);
  else if (front_size <= 40) hipLaunchKernelGGL((k_fold_small<40, 128, 16>), dim3(ncl, nb), dim3(128), 0, st, c, cls);
  else if (front_size <= 48) hipLaunchKernelGGL((k_fold_small<48, 256, 16>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
  else hipLaunchKernelGGL((k_fold_small<64, 256, 16>), dim3(ncl, nb), dim3(256), 0, st, c, cls);
}

void launch_extract_small(const Ctx& c, const int32_t* cls, int ncl, int nb, size_t lds_bytes, size_t lds_bytes_leaf,
                          int front_size, bool lesser, hipStream_t st) {
  static bool attr_set = false;
  if (!attr_set) {
    // the gathered B x B block can exceed 64 KB; gfx950 gives a block up to 160 KB
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_extract_small<512>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_extract_small<256>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  if (ncl <= 0) return;
  const int w = lesser ? 1 : 0;
  // the larger classes hold few blocks per CU (LDS), so each block runs more
  // threads: more independent outputs in flight per front
  // with phonon sources every cluster keeps its full rows (no leaf layout)
  const size_t lds = c.scat ? lds_bytes : lds_bytes_leaf;
  switch (extract_threads(front_size)) {
    case 64: hipLaunchKernelGGL((k_extract_small<64>), dim3(ncl, nb), dim3(64), lds, st, c, cls, w); break;
    case 256: hipLaunchKernelGGL((k_extract_small<256>), dim3(ncl, nb), dim3(256), lds, st, c, cls, w); break;
    default: hipLaunchKernelGGL((k_extract_small<512>), dim3(ncl, nb), dim3(512), lds, st, c, cls, w); break;
  }
}

}  // namespace ndg
