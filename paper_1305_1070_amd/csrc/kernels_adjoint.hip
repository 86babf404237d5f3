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
// factors of the fold (Section 3.2): forward substitution up the tree
// (Z_i = Y_i + sum of the children's contributions Psi_d^T Z_d), the block
// diagonal D^{-1} (the pivot inverses), and back substitution down the tree
// (X_i = D^{-1}Z_i + Psi_i X_{B_i}).  The factors are recomputed by a fresh
// fold rather than kept from the forward pass.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "kernels.hpp"

namespace ndg {

// Y = E_c: ones at (contact site a, column a) in the internal ordering.
__global__ void k_rhs_contact(Ctx c, RhsCtx r, int cc) {
  const int e = blockIdx.y;
  double2* Y = r.Y + (int64_t)e * r.n * r.m;
  const int64_t total = (int64_t)r.n * r.m;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256)
    Y[q] = cz();
  // (the ones are placed by k_rhs_contact_ones after this kernel)
}

__global__ void k_rhs_contact_ones(Ctx c, RhsCtx r, int cc) {
  const int e = blockIdx.y;
  double2* Y = r.Y + (int64_t)e * r.n * r.m;
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= c.nc[cc]) return;
  Y[(int64_t)c.cpos[cc][a] * r.m + a] = make_double2(1.0, 0.0);
}

// Y = Lambda conj(G_{:,c}) with Lambda = diag(nbar) in the caller's order.
__global__ void k_rhs_lambda(Ctx c, RhsCtx r) {
  const int e = blockIdx.y;
  const double2* G = r.Gc + (int64_t)e * r.n * r.m;
  double2* Y = r.Y + (int64_t)e * r.n * r.m;
  const int64_t total = (int64_t)r.n * r.m;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total; q += (int64_t)gridDim.x * 256) {
    const int row = (int)(q / r.m);
    const double w = r.nbar[c.perm[row]];
    const double2 g = G[q];
    Y[q] = make_double2(w * g.x, -w * g.y);
  }
}

// Forward substitution and D^{-1} for one cluster (bottom-up by levels):
// the front vector Zf (f x m) gathers the children's contributions, adds the
// cluster's rows of Y, passes V = Zf_B + Psi^T Z_I up, and stores
// D^{-1} Z_I = A_ii^{-1} Z_I in the cluster's rows of X.
__global__ void __launch_bounds__(256) k_rhs_fwd(Ctx c, RhsCtx r, const int32_t* cls) {
  __shared__ GemmSmem sm;
  const int cl = cls[blockIdx.x];
  const int e = blockIdx.y;
  const ClusterDesc d = c.cl[cl];
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  const double2* Ainv = S + d.o_ainv;
  const int m = r.m, s = d.s, b = d.b, f = d.f;
  double2* Zsl = r.Z + (int64_t)e * r.zstride;
  double2* Zf = Zsl + r.o_vec[cl];
  const double2* Y = r.Y + (int64_t)e * r.n * m;
  double2* X = r.X + (int64_t)e * r.n * m;
  const int t = threadIdx.x;
  for (int q = t; q < f * m; q += 256) Zf[q] = q < s * m ? Y[(int64_t)d.pt_off * m + q] : cz();
  __syncthreads();
  for (int kp = c.kids_ptr[cl]; kp < c.kids_ptr[cl + 1]; ++kp) {
    const int ch = c.kids[kp];
    const ClusterDesc dc = c.cl[ch];
    const double2* Zc = Zsl + r.o_vec[ch];
    const int32_t* rel = c.relmap + dc.bptr;
    for (int q = t; q < dc.b * m; q += 256) {
      const int rr = q / m, a = q - rr * m;
      double2 v = Zf[(int64_t)rel[rr] * m + a];
      const double2 u = Zc[(int64_t)(dc.s + rr) * m + a];
      v.x += u.x;
      v.y += u.y;
      Zf[(int64_t)rel[rr] * m + a] = v;
    }
    __syncthreads();
  }
  for (int i0 = 0; i0 < b; i0 += 64) {
    const int ni = min(64, b - i0);
    for (int j0 = 0; j0 < m; j0 += 64) {
      const int nj = min(64, m - j0);
      ZTile acc;
      ztile_zero(acc);
      zgemm_acc<true, false>(
          s, [&](int i, int k) { return i < ni ? Psi[(int64_t)k * b + i0 + i] : cz(); },
          [&](int k, int j) { return j < nj ? Zf[(int64_t)k * m + j0 + j] : cz(); }, acc, sm);
      ztile_store(acc, [&](int i, int j, double re, double im) {
        if (i < ni && j < nj) {
          double2 v = Zf[(int64_t)(s + i0 + i) * m + j0 + j];
          v.x += re;
          v.y += im;
          Zf[(int64_t)(s + i0 + i) * m + j0 + j] = v;
        }
      });
    }
  }
  for (int j0 = 0; j0 < m; j0 += 64) {
    const int nj = min(64, m - j0);
    ZTile acc;
    ztile_zero(acc);
    zgemm_acc<false, false>(
        s, [&](int i, int k) { return i < s ? Ainv[i * s + k] : cz(); },
        [&](int k, int j) { return j < nj ? Zf[(int64_t)k * m + j0 + j] : cz(); }, acc, sm);
    ztile_store(acc, [&](int i, int j, double re, double im) {
      if (i < s && j < nj) X[(int64_t)(d.pt_off + i) * m + j0 + j] = make_double2(re, im);
    });
  }
}

// Back substitution (top-down by levels): X_I = X_I + Psi_i X_{B_i}, the
// B_i rows gathered from the ancestors' final rows of X.
__global__ void __launch_bounds__(256) k_rhs_back(Ctx c, RhsCtx r, const int32_t* cls) {
  __shared__ GemmSmem sm;
  const int cl = cls[blockIdx.x];
  const int e = blockIdx.y;
  const ClusterDesc d = c.cl[cl];
  if (d.b == 0) return;
  double2* S = slab(c, e);
  const double2* Psi = S + d.o_psi;
  const int m = r.m, s = d.s, b = d.b;
  double2* X = r.X + (int64_t)e * r.n * m;
  const int32_t* bidx = r.bidx + d.bptr;
  for (int j0 = 0; j0 < m; j0 += 64) {
    const int nj = min(64, m - j0);
    ZTile acc;
    ztile_zero(acc);
    zgemm_acc<false, false>(
        b, [&](int i, int k) { return i < s ? Psi[(int64_t)i * b + k] : cz(); },
        [&](int k, int j) { return j < nj ? X[(int64_t)bidx[k] * m + j0 + j] : cz(); }, acc, sm);
    ztile_store(acc, [&](int i, int j, double re, double im) {
      if (i < s && j < nj) {
        double2 v = X[(int64_t)(d.pt_off + i) * m + j0 + j];
        v.x += re;
        v.y += im;
        X[(int64_t)(d.pt_off + i) * m + j0 + j] = v;
      }
    });
  }
}

// T = G_{:,c} Sigma^<_c (n x m, written over Y, which is free by now):
// 64 x 64 tiles on the FP64 matrix cores, grid = (row tiles * col tiles, nb).
__global__ void __launch_bounds__(256) k_vjp_gemm(Ctx c, RhsCtx r, int cc) {
  __shared__ GemmSmem sm;
  const int e = blockIdx.y;
  const int m = r.m;
  const int ntc = (m + 63) / 64;
  const int i0 = (blockIdx.x / ntc) * 64, j0 = (blockIdx.x % ntc) * 64;
  const int ni = min(64, r.n - i0), nj = min(64, m - j0);
  const double2* G = r.Gc + (int64_t)e * r.n * m;
  const double2* sg = c.sig_l[cc] + (int64_t)(c.e0 + e) * m * m;
  double2* T = r.Y + (int64_t)e * r.n * m;
  ZTile acc;
  ztile_zero(acc);
  zgemm_acc<false, false>(
      m, [&](int i, int k) { return i < ni ? G[(int64_t)(i0 + i) * m + k] : cz(); },
      [&](int k, int j) { return j < nj ? sg[(int64_t)k * m + j0 + j] : cz(); }, acc, sm);
  ztile_store(acc, [&](int i, int j, double re, double im) {
    if (i < ni && j < nj) T[(int64_t)(i0 + i) * m + j0 + j] = make_double2(re, im);
  });
}

// part[e][row] += 2 Im[ sum_b T[row,b] X[row,b] ]
__global__ void __launch_bounds__(256) k_vjp_accum(Ctx c, RhsCtx r, int cc) {
  const int e = blockIdx.y;
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= r.n) return;
  const int m = r.m;
  const double2* T = r.Y + ((int64_t)e * r.n + row) * m;
  const double2* X = r.X + ((int64_t)e * r.n + row) * m;
  double acc = 0.0;
  for (int bb = 0; bb < m; ++bb) {
    const double2 t = T[bb], x = X[bb];
    acc += t.x * x.y + t.y * x.x;  // Im[(t.x + i t.y)(x.x + i x.y)]
  }
  r.part[(int64_t)e * r.n + row] += 2.0 * acc;
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

void launch_rhs_contact(const Ctx& c, const RhsCtx& r, int cc, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_contact, dim3(256, nb), dim3(256), 0, st, c, r, cc);
  hipLaunchKernelGGL(k_rhs_contact_ones, dim3((c.nc[cc] + 255) / 256, nb), dim3(256), 0, st, c, r, cc);
}
void launch_rhs_lambda(const Ctx& c, const RhsCtx& r, int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_rhs_lambda, dim3(256, nb), dim3(256), 0, st, c, r);
}
void launch_rhs_fwd(const Ctx& c, const RhsCtx& r, const int32_t* cls, int ncl, int nb, hipStream_t st) {
  if (ncl > 0) hipLaunchKernelGGL(k_rhs_fwd, dim3(ncl, nb), dim3(256), 0, st, c, r, cls);
}
void launch_rhs_back(const Ctx& c, const RhsCtx& r, const int32_t* cls, int ncl, int nb, hipStream_t st) {
  if (ncl > 0) hipLaunchKernelGGL(k_rhs_back, dim3(ncl, nb), dim3(256), 0, st, c, r, cls);
}
void launch_vjp_accum(const Ctx& c, const RhsCtx& r, int cc, int nb, hipStream_t st) {
  const int tiles = ((r.n + 63) / 64) * ((r.m + 63) / 64);
  hipLaunchKernelGGL(k_vjp_gemm, dim3(tiles, nb), dim3(256), 0, st, c, r, cc);
  hipLaunchKernelGGL(k_vjp_accum, dim3((r.n + 255) / 256, nb), dim3(256), 0, st, c, r, cc);
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

}  // namespace ndg
