// Density and its gradient with respect to the on-site potential.
//
// Density: n_i = sum_E c_E (-i G^<_ii(E)), accumulated per site over the
// energies of a batch in a fixed order (deterministic).
//
// Gradient (vector-Jacobian product for a cotangent nbar on n):
//   dA/dV_k = -e_k e_k^T  =>  dG^< = G e_k e_k^T G^< + G^< e_k e_k^T G^+, so
//   Vbar_k = sum_E c_E 2 Im[(G^< Lambda G^r)_kk],   Lambda = diag(nbar).
// Without phonons G^< = sum_c G_{:,c} Sigma^<_c G_{:,c}^+ over the contacts,
// and with G = G^T
//   (G^< Lambda G)_kk = sum_c [G_{k,c} Sigma^<_c X_c(k,:)^T],
//   X_c = A^{-1} (Lambda conj(G_{:,c})).
// Both G_{:,c} = A^{-1} E_c and X_c are multi-right-hand-side solves with the
// factors of the fold (Section 3.2), the columns of all contacts forming one
// right-hand side: forward substitution up the tree (Z_i = Y_i + sum of the
// children's contributions Psi_d^T Z_d), then back substitution down the tree
// with the pivot inverses applied in the same step (X_i = A_ii^{-1} Z_i +
// Psi_i X_{B_i}).  The right-hand sides Y are formed where the forward
// substitution reads them (rhs_y) and never stored.  The factors are
// recomputed by a fresh fold rather than kept from the forward pass.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.hpp"
#include "kernels.hpp"

namespace ndg {

// Right-hand side entry Y[row][a] (internal row order; the columns of all
// contacts side by side): the unit columns E_c in the first solve,
// Lambda conj(G_{:,c}) with Lambda = diag(nbar) (caller's order) in the
// second; formed where the forward substitution reads it, never stored.
__device__ inline double2 rhs_y(const Ctx& c, const RhsCtx& r, int e, int row, int a) {
  if (r.ymode == 0) return make_double2(r.cinv[row] == a ? 1.0 : 0.0, 0.0);
  const double w = r.nbar[c.perm[row]];
  const double2 g = r.Gc[((int64_t)e * r.n + row) * r.m + a];
  return make_double2(w * g.x, -w * g.y);
}

// Lane layout of a 64 x 64 FP64 matrix-core tile (TileShape<64>): lane l,
// block (mm, n), register rr hold row wr + 16 mm + l/16 + 4 rr and column
// wc + 16 n + l%16 of the tile.
struct TileLanes {
  using T = TileShape<64>;
  int lane, wr, wc;
  __device__ TileLanes(int t) : lane(t & 63) {
    const int w = t >> 6;
    wr = (w / T::WN) * (64 / T::WM);
    wc = (w % T::WN) * (64 / T::WN);
  }
  __device__ int row(int mm, int rr) const { return wr + mm * 16 + (lane >> 4) + 4 * rr; }
  __device__ int col(int n) const { return wc + n * 16 + (lane & 15); }
};

// Clusters with s <= kRhsSmallS, b <= kRhsSmallB and s b <= kRhsSmallSB (the
// leaves and the separators of the lower heights, most clusters) are solved by one
// wavefront each: lane = right-hand-side column (a row of 64 columns is 1 KB
// contiguous), Psi and A_ii^{-1} staged in LDS sized per height by the
// launch, the short products on the vector units.  Matrix tiles of 64 x 64
// would be mostly padding there.
constexpr int kRhsS = kRhsSmallS;
__device__ inline bool rhs_small(const ClusterDesc& d) {
  return d.s <= kRhsSmallS && d.b <= kRhsSmallB && d.s * d.b <= kRhsSmallSB;
}

__global__ void __launch_bounds__(64) k_rhs_fwd_small(Ctx c, RhsCtx r, const int32_t* cls) {
  extern __shared__ double2 psi[];  // s x b
  __shared__ int64_t kid_inv[kMaxKids], kid_z[kMaxKids];
  const int cl = cls[blockIdx.x];
  const int e = blockIdx.y;
  const ClusterDesc d = c.cl[cl];
  if (!rhs_small(d)) return;  // k_rhs_fwd
  const double2* Psi = slab(c, e) + d.o_psi;
  const int m = r.m, s = d.s, b = d.b;
  const double2* Zsl = r.Z + (int64_t)e * r.zstride;
  double2* Zf = r.Z + (int64_t)e * r.zstride + r.o_vec[cl];
  const int t = threadIdx.x;
  const int k0 = c.kids_ptr[cl], nk = c.kids_ptr[cl + 1] - k0;
  for (int q = t; q < nk; q += 64) {
    const int ch = c.kids[k0 + q];
    const ClusterDesc& dc = c.cl[ch];
    kid_inv[q] = dc.o_pinv;
    kid_z[q] = r.o_vec[ch] + (int64_t)dc.s * m;
  }
  for (int q = t; q < s * b; q += 64) psi[q] = Psi[q];  // row k = I index, column i = B index
  __syncthreads();
  for (int a0 = 0; a0 < m; a0 += 64) {
    const int a = a0 + t;
    const bool on = a < m;
    double2 zi[kRhsS];
#pragma unroll
    for (int x = 0; x < kRhsS; ++x) {
      zi[x] = cz();
      if (x < s) {
        double2 v = on ? rhs_y(c, r, e, d.pt_off + x, a) : cz();
        for (int kq = 0; kq < nk; ++kq) {
          const int ci = c.pinv[kid_inv[kq] + x];
          if (ci >= 0 && on) {
            const double2 u = Zsl[kid_z[kq] + (int64_t)ci * m + a];
            v.x += u.x;
            v.y += u.y;
          }
        }
        zi[x] = v;
        // a leaf's Z_I is its right-hand side: the back substitution forms it again
        if (on && nk > 0) Zf[(int64_t)x * m + a] = v;
      }
    }
    for (int i = 0; i < b; ++i) {
      double2 v = cz();
      for (int kq = 0; kq < nk; ++kq) {
        const int ci = c.pinv[kid_inv[kq] + s + i];
        if (ci >= 0 && on) {
          const double2 u = Zsl[kid_z[kq] + (int64_t)ci * m + a];
          v.x += u.x;
          v.y += u.y;
        }
      }
#pragma unroll
      for (int k = 0; k < kRhsS; ++k)
        if (k < s) cmac(v, psi[k * b + i], zi[k]);  // (Psi^T Z_I)_i = sum_k Psi[k][i] Z_I[k]
      if (on) Zf[(int64_t)(s + i) * m + a] = v;
    }
  }
}

__global__ void __launch_bounds__(64) k_rhs_back_small(Ctx c, RhsCtx r, const int32_t* cls) {
  extern __shared__ double2 dsm[];  // Psi (s x b), A_ii^{-1} (s x s), B_i positions (b)
  const int cl = cls[blockIdx.x];
  const int e = blockIdx.y;
  const ClusterDesc d = c.cl[cl];
  if (!rhs_small(d)) return;  // k_rhs_back
  double2* S = slab(c, e);
  const int m = r.m, s = d.s, b = d.b;
  double2* psi = dsm;
  double2* ainv = dsm + s * b;
  int32_t* bix = reinterpret_cast<int32_t*>(ainv + s * s);
  const bool leaf = c.kids_ptr[cl + 1] == c.kids_ptr[cl];  // Z_I not stored (k_rhs_fwd_small)
  const double2* Zf = r.Z + (int64_t)e * r.zstride + r.o_vec[cl];
  double2* X = r.X + (int64_t)e * r.n * m;
  const int t = threadIdx.x;
  for (int q = t; q < s * b; q += 64) psi[q] = S[d.o_psi + q];
  for (int q = t; q < s * s; q += 64) ainv[q] = S[d.o_ainv + q];
  for (int q = t; q < b; q += 64) bix[q] = r.bidx[d.bptr + q];
  __syncthreads();
  for (int a0 = 0; a0 < m; a0 += 64) {
    const int a = a0 + t;
    const bool on = a < m;
    double2 xo[kRhsS];
#pragma unroll
    for (int i = 0; i < kRhsS; ++i) xo[i] = cz();
    // one input row at a time: only the outputs stay in registers
    for (int k = 0; k < s; ++k) {
      const double2 z = !on ? cz() : leaf ? rhs_y(c, r, e, d.pt_off + k, a) : Zf[(int64_t)k * m + a];
#pragma unroll
      for (int i = 0; i < kRhsS; ++i)
        if (i < s) cmac(xo[i], ainv[i * s + k], z);
    }
    for (int k = 0; k < b; ++k) {
      const double2 xb = on ? X[(int64_t)bix[k] * m + a] : cz();
#pragma unroll
      for (int i = 0; i < kRhsS; ++i)
        if (i < s) cmac(xo[i], psi[i * b + k], xb);
    }
#pragma unroll
    for (int i = 0; i < kRhsS; ++i)
      if (i < s && on) X[(int64_t)(d.pt_off + i) * m + a] = xo[i];
  }
}

// Forward substitution for one cluster (bottom-up by levels).  The cluster's
// rows of its front vector, Z_I = Y_I + the children's contributions to I,
// are gathered in one pass; the rows passed up to the parent,
// Z_B = the children's contributions to B + Psi^T Z_I, are formed in the
// matrix-core tile (children gathered through their index maps into the
// accumulators, then the product on top).  Every row is written once; the
// block diagonal D^{-1} is applied by the back substitution.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_rhs_fwd(Ctx c, RhsCtx r, const int32_t* cls) {
  __shared__ GemmSmem sm;
  __shared__ int64_t kid_inv[kMaxKids], kid_z[kMaxKids];
  const int cl = cls[blockIdx.x];
  const int e = blockIdx.y;
  const ClusterDesc d = c.cl[cl];
  if (rhs_small(d)) return;  // k_rhs_fwd_small
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  const int m = r.m, s = d.s, b = d.b;
  const double2* Zsl = r.Z + (int64_t)e * r.zstride;
  double2* Zf = r.Z + (int64_t)e * r.zstride + r.o_vec[cl];
  const int t = threadIdx.x;
  const int k0 = c.kids_ptr[cl], nk = c.kids_ptr[cl + 1] - k0;
  for (int q = t; q < nk; q += 256) {
    const int ch = c.kids[k0 + q];
    const ClusterDesc& dc = c.cl[ch];
    kid_inv[q] = dc.o_pinv;                             // parent front position -> child B index
    kid_z[q] = r.o_vec[ch] + (int64_t)dc.s * m;         // the child's B rows
  }
  __syncthreads();
  // four entries per thread at a time: each round of dependent loads
  // (right-hand side, children's maps, their rows) issued for all four
  // before any entry is stored
  const int nq = s * m;
  for (int q0 = t; q0 < nq; q0 += 4 * 256) {
    int xs[4], as[4];
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int q = min(q0 + u * 256, nq - 1);  // past the end: a repeat, not stored
      xs[u] = q / m;
      as[u] = q - xs[u] * m;
      v[u] = rhs_y(c, r, e, d.pt_off + xs[u], as[u]);
    }
    for (int kq = 0; kq < nk; ++kq) {
      int ci[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) ci[u] = c.pinv[kid_inv[kq] + xs[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (ci[u] >= 0) {
          const double2 z = Zsl[kid_z[kq] + (int64_t)ci[u] * m + as[u]];
          v[u].x += z.x;
          v[u].y += z.y;
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (q0 + u * 256 < nq) Zf[q0 + u * 256] = v[u];
  }
  if (b == 0) return;  // the root passes nothing up
  __threadfence_block();
  __syncthreads();  // Z_I complete: the product below reads it
  using T = TileShape<64>;
  const TileLanes L(t);
  for (int i0 = 0; i0 < b; i0 += 64) {
    const int ni = min(64, b - i0);
    for (int j0 = 0; j0 < m; j0 += 64) {
      const int nj = min(64, m - j0);
      ZTile acc;
      ztile_zero(acc);
      for (int kq = 0; kq < nk; ++kq) {
        const int32_t* inv = c.pinv + kid_inv[kq];
        const double2* Zc = Zsl + kid_z[kq];
        int ri[T::MB][4];
#pragma unroll
        for (int mm = 0; mm < T::MB; ++mm)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = L.row(mm, rr);
            ri[mm][rr] = i < ni ? inv[s + i0 + i] : -1;
          }
#pragma unroll
        for (int mm = 0; mm < T::MB; ++mm)
#pragma unroll
          for (int n = 0; n < T::NB; ++n)
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
              const int j = L.col(n);
              if (ri[mm][rr] >= 0 && j < nj) {
                const double2 u = Zc[(int64_t)ri[mm][rr] * m + j0 + j];
                acc.re[mm][n][rr] += u.x;
                acc.im[mm][n][rr] += u.y;
              }
            }
      }
      zgemm_acc_t<64, true, false, true>(
          s, [&](int i, int k) { return i < ni ? Psi[(int64_t)k * b + i0 + i] : cz(); },
          [&](int k, int j) { return j < nj ? Zf[(int64_t)k * m + j0 + j] : cz(); }, acc, sm, ni, nj);
      ztile_store_t<64>(acc, [&](int i, int j, double re, double im) {
        if (i < ni && j < nj) Zf[(int64_t)(s + i0 + i) * m + j0 + j] = make_double2(re, im);
      });
    }
  }
}

// Back substitution (top-down by levels): X_I = A_ii^{-1} Z_I + Psi_i X_{B_i},
// both products into one tile, the B_i rows gathered from the ancestors'
// final rows of X; the cluster's rows of X are written once.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_rhs_back(Ctx c, RhsCtx r, const int32_t* cls) {
  __shared__ GemmSmem sm;
  const int cl = cls[blockIdx.x];
  const int e = blockIdx.y;
  const ClusterDesc d = c.cl[cl];
  if (rhs_small(d)) return;  // k_rhs_back_small
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  const double2* Ainv = S + d.o_ainv;
  const int m = r.m, s = d.s, b = d.b;
  const double2* Zf = r.Z + (int64_t)e * r.zstride + r.o_vec[cl];
  double2* X = r.X + (int64_t)e * r.n * m;
  const int32_t* bidx = r.bidx + d.bptr;
  for (int j0 = 0; j0 < m; j0 += 64) {
    const int nj = min(64, m - j0);
    ZTile acc;
    ztile_zero(acc);
    zgemm_acc_t<64, false, false, true>(
        s, [&](int i, int k) { return i < s ? Ainv[i * s + k] : cz(); },
        [&](int k, int j) { return j < nj ? Zf[(int64_t)k * m + j0 + j] : cz(); }, acc, sm, s, nj);
    if (b > 0)
      zgemm_acc_t<64, false, false, true>(
          b, [&](int i, int k) { return i < s ? Psi[(int64_t)i * b + k] : cz(); },
          [&](int k, int j) { return j < nj ? X[(int64_t)bidx[k] * m + j0 + j] : cz(); }, acc, sm, s, nj);
    ztile_store_t<64>(acc, [&](int i, int j, double re, double im) {
      if (i < s && j < nj) X[(int64_t)(d.pt_off + i) * m + j0 + j] = make_double2(re, im);
    });
  }
}

// part[e][row] += 2 Im[ sum_a T[row][a] X[row][a] ],  T = G_{:,c} Sigma^<_c,
// over contact c's block of columns [off, off + n_c) of G and X.
// One block per 64 rows: each 64-column tile of T is formed on the matrix
// cores and consumed in registers (never stored); the row sums are reduced
// across the lanes of a row and the two column halves of the tile, column
// tiles in order (deterministic).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_vjp(Ctx c, RhsCtx r, int cc, int off) {
  __shared__ GemmSmem sm;
  using T = TileShape<64>;
  __shared__ double rowsum[T::WN][64];
  const int e = blockIdx.y;
  const int m = r.m;             // row stride: all contacts' columns
  const int mc = sel2(c.nc, cc);  // this contact's columns [off, off + mc)
  const int i0 = blockIdx.x * 64;
  const int ni = min(64, r.n - i0);
  const double2* G = r.Gc + (int64_t)e * r.n * m + off;
  const double2* sg = sel2(c.sig_l, cc) + (int64_t)(c.e0 + e) * mc * mc;
  const double2* X = r.X + (int64_t)e * r.n * m + off;
  const int t = threadIdx.x;
  const TileLanes L(t);
  double rs[T::MB][4];
#pragma unroll
  for (int mm = 0; mm < T::MB; ++mm)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) rs[mm][rr] = 0.0;
  for (int j0 = 0; j0 < mc; j0 += 64) {
    const int nj = min(64, mc - j0);
    ZTile acc;
    ztile_zero(acc);
    zgemm_acc_t<64, false, false, true>(
        mc, [&](int i, int k) { return i < ni ? G[(int64_t)(i0 + i) * m + k] : cz(); },
        [&](int k, int j) { return j < nj ? sg[(int64_t)k * mc + j0 + j] : cz(); }, acc, sm, ni, nj);
#pragma unroll
    for (int mm = 0; mm < T::MB; ++mm)
#pragma unroll
      for (int n = 0; n < T::NB; ++n)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int i = L.row(mm, rr), j = L.col(n);
          if (i < ni && j < nj) {
            const double2 x = X[(int64_t)(i0 + i) * m + j0 + j];
            // Im[(t.x + i t.y)(x.x + i x.y)]
            rs[mm][rr] += (double)acc.re[mm][n][rr] * x.y + (double)acc.im[mm][n][rr] * x.x;
          }
        }
  }
  // the 16 lanes of a row (same lane / 16) hold its columns
#pragma unroll
  for (int mm = 0; mm < T::MB; ++mm)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      double v = rs[mm][rr];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off);
      if ((L.lane & 15) == 0) rowsum[(t >> 6) % T::WN][L.row(mm, rr)] = v;
    }
  __syncthreads();
  if (t < ni) {
    double v = 0.0;
#pragma unroll
    for (int h = 0; h < T::WN; ++h) v += rowsum[h][t];
    r.part[(int64_t)e * r.n + i0 + t] += 2.0 * v;
  }
}

__global__ void k_zero(double* p, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

// Vbar[perm[row]] += sum_e cE[e] part[e][row], energies in order.
__global__ void k_vjp_reduce(Ctx c, RhsCtx r, int nb, const double* cE, double* vbar) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= r.n) return;
  double acc = 0.0;
  for (int e = 0; e < nb; ++e) acc += cE[c.e0 + e] * r.part[(int64_t)e * r.n + row];
  vbar[c.perm[row]] += acc;
}

// density[perm[row]] += sum_e cE[e] Re(-i G^<_rr), energies in order.
__global__ void k_density(Ctx c, int nb, const double* cE, double* dens) {
  const int q = blockIdx.x * 256 + threadIdx.x;  // site in the caller's order
  if (q >= c.n) return;
  const int64_t ol = c.sdiag[q].ol;
  double acc = 0.0;
  for (int e = 0; e < nb; ++e) {
    const double2 gl = (c.ws + (int64_t)e * c.stride)[ol];
    acc += cE[c.e0 + e] * gl.y;  // Re(-i (x + i y)) = y
  }
  dens[q] += acc;
}

// Both variants over all clusters of a height; each skips the other's.
// small_lds: the small variant's dynamic LDS for this height (0: no small
// cluster), big: whether the height has a cluster for the tiled variant.
void launch_rhs_fwd(const Ctx& c, const RhsCtx& r, const int32_t* cls, int ncl, int nb, size_t small_lds,
                    bool big, hipStream_t st) {
  if (ncl <= 0) return;
  if (small_lds) hipLaunchKernelGGL(k_rhs_fwd_small, dim3(ncl, nb), dim3(64), small_lds, st, c, r, cls);
  if (big) hipLaunchKernelGGL(k_rhs_fwd, dim3(ncl, nb), dim3(256), 0, st, c, r, cls);
}
void launch_rhs_back(const Ctx& c, const RhsCtx& r, const int32_t* cls, int ncl, int nb, size_t small_lds,
                     bool big, hipStream_t st) {
  if (ncl <= 0) return;
  if (small_lds) hipLaunchKernelGGL(k_rhs_back_small, dim3(ncl, nb), dim3(64), small_lds, st, c, r, cls);
  if (big) hipLaunchKernelGGL(k_rhs_back, dim3(ncl, nb), dim3(256), 0, st, c, r, cls);
}
void launch_vjp_accum(const Ctx& c, const RhsCtx& r, int cc, int off, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_vjp, dim3((r.n + 63) / 64, nb), dim3(256), 0, st, c, r, cc, off);
}
void launch_zero(double* p, int64_t count, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_zero, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count);
}
void launch_vjp_reduce(const Ctx& c, const RhsCtx& r, int nb, const double* cE, double* vbar, hipStream_t st) {
  hipLaunchKernelGGL(k_vjp_reduce, dim3((r.n + 255) / 256), dim3(256), 0, st, c, r, nb, cE, vbar);
}
void launch_density(const Ctx& c, int nb, const double* cE, double* dens, hipStream_t st) {
  hipLaunchKernelGGL(k_density, dim3((c.n + 255) / 256), dim3(256), 0, st, c, nb, cE, dens);
}

// ---------------------------------------------------------------------------
// Static partials buffer of ndg_density_vjp_noalloc (for callers that cannot
// allocate): 4 Mi doubles (32 MiB), one copy per GPU, held until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol): its address on each device comes from
// hipGetSymbolAddress, taken once per device with that device current.  Calls
// that overlap on one GPU race on this buffer.
constexpr int64_t kNoAllocDoubles = int64_t(4) << 20;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

double* noalloc_scratch(int device, int64_t* capacity) {
  static std::mutex mu;
  static double* addr[kNoAllocDevices] = {};
  *capacity = 0;
  if (device < 0 || device >= kNoAllocDevices) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != device && hipSetDevice(device) != hipSuccess) return nullptr;
    void* ptr = nullptr;
    const hipError_t rc = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (rc != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    addr[device] = static_cast<double*>(ptr);
  }
  *capacity = kNoAllocDoubles;
  return addr[device];
}

}  // namespace ndg
