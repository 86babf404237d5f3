// G^< source for a Sigma^< on every cluster (diagonal phonon self-energy),
// Section 3.2 "Computation of blocks for G^<", steps 1-3, with P_i the set of
// ALL ancestors of cluster i as the paper defines it.
//
// Without phonons Sigma^< sits on the contacts and the source is formed on
// the contacts' ancestor chains only.  With a diagonal Sigma^<_ph every row
// of N = Sigma^< (G^(0))+ is nonzero, and the fold of N carries each
// cluster's row block across all of its ancestors' points, not only the
// coupled ones B_i (a cluster's source reaches an ancestor it is not coupled
// to through the ancestors in between).  Three passes, each over one height
// per launch:
//   k_anc_g   top-down:  G_{i,Anc} = Psi_i G_{B_i,Anc}   (the paper's G^(0)
//             over every (cluster, ancestor) pair; G_{B,Anc} is read from
//             the ancestors' rows of this pass, directly or transposed,
//             G^r being complex symmetric), G_ii copied from the G^r
//             extraction;
//   k_anc_n   bottom-up: N_i = Sigma^<_ph,i conj(G_{i,frame})
//             + sum over descendants d with B_d meeting i of
//               Psi_{d,i}^T N_{d, frame of i}
//             (the fold N_jk += Psi_ij^T N_ik, gathered by the receiving
//             cluster: no contribution blocks are stored, no atomics);
//   k_anc_p0  P_init = A_ii^{-1} N_{i, [i, B_i]}, written into the G^< front
//             (added to the contact chains' part where the cluster lies on
//             one, since the source is linear in Sigma^<).
// The extraction of G^< then runs unchanged with a source on every cluster.
//
// Also here: the self-consistent Born update of local elastic scattering
// (k_scba_mix, k_scba_max) and the terminal current spectral density per
// contact (k_current), which read the outputs and stored rows of a solve.
#include "device_common.hpp"

#include <algorithm>

namespace ndg {

namespace {

// Frame tables of one cluster in LDS: per chain index a (0 = the cluster),
// the owner's row block offset and row length, and the frame offsets ao.
struct FrameLds {
  int64_t og[kMaxAncestors + 1];
  int32_t gg[kMaxAncestors + 1];
  int32_t ao[kMaxAncestors + 2];
};

__device__ inline void load_frame(const ScatCtx& x, const ScatDesc& sd, FrameLds& fr) {
  const int32_t* tab = x.atab + sd.tab;
  for (int q = threadIdx.x; q <= sd.D; q += blockDim.x) {
    const ScatDesc a = x.sd[tab[q]];
    fr.og[q] = a.o_g;
    fr.gg[q] = a.g;
  }
  for (int q = threadIdx.x; q < sd.D + 2; q += blockDim.x) fr.ao[q] = tab[sd.D + 1 + q];
}

}  // namespace

// G_{i, Anc_i} = Psi_i G_{B_i, Anc_i}, one 64-column tile of the frame per
// block; the tile's columns inside the cluster's own points take G_ii from
// the G^r extraction.  Entry (x, y) of G_{B,Anc}, x in the frame's cluster
// a_x and y in a_y: the rows of the lower of the two (G(x, y) in a_x's rows
// when a_y >= a_x, else G(y, x) in a_y's rows).  A leaf's rows are gathered
// by nobody and its N has no descendants' part, so a leaf stores
// N_i = Sigma^<_ph,i conj(G) at once (k_anc_n skips the leaves); LEAF
// launches (height 1) hold only leaves.
template <int TM, bool LEAF>
__device__ __forceinline__ void anc_g_body(const Ctx& c, const ScatCtx& x, const ColItem* items) {
  __shared__ GemmSmemR<TM> sm;
  __shared__ FrameLds fr;
  __shared__ int32_t col_a[64];
  __shared__ double2 sig_row[kClusterRows];
  const WorkIdx wk = xcd_work();
  const ColItem it = items[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[it.cl];
  const ScatDesc sd = x.sd[it.cl];
  double2* S = slab(c, e);
  double2* X = x.ws + (int64_t)e * x.stride;
  const int s = d.s, b = d.b, f = d.f, g = sd.g, D = sd.D;
  const int j0 = it.tc * 64, nj = min(64, g - j0);
  load_frame(x, sd, fr);
  if (LEAF && threadIdx.x < s) sig_row[threadIdx.x] = c.sig_l_ph[(int64_t)(eb + e) * c.n + c.perm[d.pt_off + threadIdx.x]];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int y = j0 + threadIdx.x;
    int a = 0;
    while (a < D && fr.ao[a + 1] <= y) ++a;
    col_a[threadIdx.x] = a;
  }
  __syncthreads();
  const double2* Psi = S + d.o_psi;
  const double2* Gf = S + d.o_fg;
  const BPos* bp = x.bpos + d.bptr;
  double2* Gi = X + sd.o_g;
  ZTile acc;
  ztile_zero(acc);
  if (j0 + nj > s)
    zgemm_acc_t<TM, false, false, true, TM, true>(
        b, [&](int i, int k) { return i < s ? Psi[(int64_t)i * b + k] : cz(); },
        [&](int k, int j) {
          const int y = j0 + j;
          if (j >= nj || y < s) return cz();
          const BPos u = bp[k];
          const int ay = col_a[j];
          int64_t addr;
          if (ay >= u.a) addr = fr.og[u.a] + (int64_t)(u.col - fr.ao[u.a]) * fr.gg[u.a] + (y - fr.ao[u.a]);
          else addr = fr.og[ay] + (int64_t)(y - fr.ao[ay]) * fr.gg[ay] + (u.col - fr.ao[ay]);
          return X[addr];
        },
        acc, sm, s, nj);
  ztile_store_t<TM>(acc, [&](int i, int j, double re, double im) {
    const int y = j0 + j;
    if (i < s && j < nj) {
      double2 v = y < s ? Gf[(int64_t)i * f + y] : make_double2(re, im);
      if constexpr (LEAF) {
        const double2 sg = sig_row[i];
        v = make_double2(sg.x * v.x + sg.y * v.y, sg.y * v.x - sg.x * v.y);   // sigma conj(G)
      }
      Gi[(int64_t)i * g + y] = v;
    }
  });
}

template <int TM>
__global__ void __launch_bounds__(256) k_anc_g(Ctx c, ScatCtx x, const ColItem* items) {
  anc_g_body<TM, false>(c, x, items);
}
// the leaves' epilogue holds more registers: the hint keeps the 16-row
// tiles (most leaves) at seven waves per SIMD
template <int TM, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE)))
k_anc_g_leaf(Ctx c, ScatCtx x, const ColItem* items) {
  anc_g_body<TM, true>(c, x, items);
}

// The N fold's product for one tile: the sum over the feeding descendants d
// of A_d (TM x s_d) times B_d (s_d x 64), A_d(i, r) = Psi_d[r][u(i)] (the
// B_d column of point i, 0 where i is not in B_d), B_d(r, j) = the entry of
// N_d's row r at column j of the tile.  The descendants' rows run as one
// stream of 16-deep K chunks (the last chunk of each descendant cut to its
// live 4-deep steps), and the operands of the next chunk, which may be the
// next descendant's first, are loaded into registers while the matrix
// cores work on the current one: most descendants hold a single chunk, so
// a product per descendant would wait on every first load.
struct Feed {
  const double2* psi;
  const double2* n;
  const int32_t* um;
  int bd, gd, sd;
  int64_t coff;
};

template <int TM>
__device__ __forceinline__ void anc_n_product(const Ctx& c, const ScatCtx& x, const ScatDesc& sd,
                                              const double2* S, const double2* X, int s, int j0, int nj,
                                              ZTile& acc, GemmSmemR<TM>& sm) {
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
  auto feed = [&](int q) {
    const LkItem L = x.lk[q];
    const ClusterDesc dd = c.cl[L.d];
    const ScatDesc sdd = x.sd[L.d];
    return Feed{S + dd.o_psi, X + sdd.o_g, x.umap + L.map, dd.b, sdd.g, dd.s, (int64_t)L.col + j0};
  };
  double2 pa[TM / 16], pb[4];
  auto load = [&](const Feed& f, int r0) {
#pragma unroll
    for (int q = 0; q < TM / 16; ++q) {
      const int idx = t + 256 * q, i = idx % TM, kk = idx / TM;
      const int u = (i < s && r0 + kk < f.sd) ? f.um[i] : -1;
      pa[q] = u >= 0 ? f.psi[(int64_t)(r0 + kk) * f.bd + u] : cz();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = t + 256 * q, j = idx & 63, kk = idx >> 6;
      pb[q] = (j < nj && r0 + kk < f.sd) ? f.n[(int64_t)(r0 + kk) * f.gd + f.coff + j] : cz();
    }
  };
  int q = sd.lk0;
  if (q >= sd.lk1) return;
  Feed cur = feed(q);
  int r0 = 0;
  load(cur, 0);
  while (true) {
#pragma unroll
    for (int qq = 0; qq < TM / 16; ++qq) {
      const int idx = t + 256 * qq, i = idx % TM, kk = idx / TM;
      sm.ar[i][kk] = pa[qq].x;
      sm.ai[i][kk] = pa[qq].y;
    }
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
      const int idx = t + 256 * qq, j = idx & 63, kk = idx >> 6;
      sm.br[kk][j] = pb[qq].x;
      sm.bi[kk][j] = pb[qq].y;
    }
    __syncthreads();
    const int kend = min(KC, cur.sd - r0);
    int nr0 = r0 + KC, nq = q;
    Feed nxt = cur;
    if (nr0 >= cur.sd) {
      nq = q + 1;
      nr0 = 0;
      if (nq < sd.lk1) nxt = feed(nq);
    }
    const bool more = nq < sd.lk1;
    if (more) load(nxt, nr0);
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      if (k4 >= kend) break;
      const int kq = k4 + (lane >> 4);
      double are[2], aim[2], bre[2], bim[2];
#pragma unroll
      for (int m = 0; m < T::MB; ++m) {
        const int i = wr + m * 16 + (lane & 15);
        are[m] = sm.ar[i][kq];
        aim[m] = sm.ai[i][kq];
      }
#pragma unroll
      for (int n = 0; n < T::NB; ++n) {
        const int j = wc + n * 16 + (lane & 15);
        bre[n] = sm.br[kq][j];
        bim[n] = sm.bi[kq][j];
      }
#pragma unroll
      for (int m = 0; m < T::MB; ++m)
#pragma unroll
        for (int n = 0; n < T::NB; ++n) {
          acc.re[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[m], bre[n], acc.re[m][n], 0, 0, 0);
          acc.re[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(-aim[m], bim[n], acc.re[m][n], 0, 0, 0);
          acc.im[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[m], bim[n], acc.im[m][n], 0, 0, 0);
          acc.im[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[m], bre[n], acc.im[m][n], 0, 0, 0);
        }
    }
    __syncthreads();
    if (!more) break;
    cur = nxt;
    r0 = nr0;
    q = nq;
  }
}

// N_i over one 64-column tile of the frame.  The own term Sigma^<_ph conj(G)
// reads the G^(0) entry that N_i replaces (same element, same thread).
// An explicit occupancy target: left to itself the compiler keeps the
// accumulators in AGPRs and runs the 64-row tiles at two wavefronts per SIMD.
template <int TM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM == 64 ? 3 : 4)))
k_anc_n(Ctx c, ScatCtx x, const ColItem* items) {
  __shared__ GemmSmemR<TM> sm;
  __shared__ double2 sig_row[kClusterRows];
  const WorkIdx wk = xcd_work();
  const ColItem it = items[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[it.cl];
  const ScatDesc sd = x.sd[it.cl];
  const double2* S = slab(c, e);
  double2* X = x.ws + (int64_t)e * x.stride;
  const int s = d.s, g = sd.g;
  const int j0 = it.tc * 64, nj = min(64, g - j0);
  if (threadIdx.x < s) sig_row[threadIdx.x] = c.sig_l_ph[(int64_t)(eb + e) * c.n + c.perm[d.pt_off + threadIdx.x]];
  __syncthreads();
  ZTile acc;
  ztile_zero(acc);
  anc_n_product<TM>(c, x, sd, S, X, s, j0, nj, acc, sm);
  double2* Ni = X + sd.o_g;
  ztile_store_t<TM>(acc, [&](int i, int j, double re, double im) {
    if (i < s && j < nj) {
      const int64_t pos = (int64_t)i * g + j0 + j;
      const double2 gv = Ni[pos];
      const double2 sg = sig_row[i];
      re += sg.x * gv.x + sg.y * gv.y;   // sigma conj(G)
      im += sg.y * gv.x - sg.x * gv.y;
      Ni[pos] = make_double2(re, im);
    }
  });
}

// P_init = A_ii^{-1} N_{i,[i, B_i]} into the cluster's rows of the G^< front.
template <int TM>
__global__ void __launch_bounds__(256) k_anc_p0(Ctx c, ScatCtx x, const int32_t* cls) {
  __shared__ GemmSmemR<TM> sm;
  const WorkIdx wk = xcd_work();
  const int cl = cls[wk.item];
  const int e = wk.e;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const ClusterDesc d = c.cl[cl];
  const ScatDesc sd = x.sd[cl];
  double2* S = slab(c, e);
  const double2* Ni = x.ws + (int64_t)e * x.stride + sd.o_g;
  const double2* Ainv = S + d.o_ainv;
  double2* FP = S + d.o_fp;
  const BPos* bp = x.bpos + d.bptr;
  const int s = d.s, f = d.f, g = sd.g;
  const bool add = d.chain_mask != 0;
  for (int j0 = 0; j0 < f; j0 += 64) {
    const int nj = min(64, f - j0);
    ZTile acc;
    ztile_zero(acc);
    zgemm_acc_t<TM, false, false, true, TM, true>(
        s, [&](int i, int k) { return i < s ? Ainv[i * s + k] : cz(); },
        [&](int k, int j) {
          if (j >= nj) return cz();
          const int cc = j0 + j;
          const int col = cc < s ? cc : bp[cc - s].col;
          return Ni[(int64_t)k * g + col];
        },
        acc, sm, s, nj);
    ztile_store_t<TM>(acc, [&](int i, int j, double re, double im) {
      if (i < s && j < nj) {
        double2* p = FP + (int64_t)i * f + j0 + j;
        if (add) {
          const double2 v = *p;
          re += v.x;
          im += v.y;
        }
        *p = make_double2(re, im);
      }
    });
  }
}

// Self-consistent Born update (local elastic scattering): per (energy, site)
// S' = d0 G_kk for the retarded and lesser self-energies, S mixed towards S',
// and per block the largest change and the largest new value; the maxima
// are combined by k_scba_max (order-independent, so deterministic).
__global__ void __launch_bounds__(256) k_scba_mix(const double2* dgr, const double2* dgl, double2* sr, double2* sl,
                                                  int64_t count, double d0, double mix, double* part) {
  __shared__ double rd[256], rs[256];
  double dmax = 0.0, smax = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < count; q += (int64_t)gridDim.x * 256) {
    const double2 gr = dgr[q], gl = dgl[q], o_r = sr[q], o_l = sl[q];
    const double2 nr = make_double2(d0 * gr.x, d0 * gr.y), nl = make_double2(d0 * gl.x, d0 * gl.y);
    dmax = fmax(dmax, fmax(hypot(nr.x - o_r.x, nr.y - o_r.y), hypot(nl.x - o_l.x, nl.y - o_l.y)));
    smax = fmax(smax, fmax(hypot(nr.x, nr.y), hypot(nl.x, nl.y)));
    sr[q] = make_double2((1.0 - mix) * o_r.x + mix * nr.x, (1.0 - mix) * o_r.y + mix * nr.y);
    sl[q] = make_double2((1.0 - mix) * o_l.x + mix * nl.x, (1.0 - mix) * o_l.y + mix * nl.y);
  }
  rd[threadIdx.x] = dmax;
  rs[threadIdx.x] = smax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + w]);
      rs[threadIdx.x] = fmax(rs[threadIdx.x], rs[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rd[0];
    part[2 * blockIdx.x + 1] = rs[0];
  }
}

__global__ void __launch_bounds__(256) k_scba_max(const double* part, int nblk, double* out) {
  __shared__ double rd[256], rs[256];
  double dmax = 0.0, smax = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 256) {
    dmax = fmax(dmax, part[2 * q]);
    smax = fmax(smax, part[2 * q + 1]);
  }
  rd[threadIdx.x] = dmax;
  rs[threadIdx.x] = smax;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + w]);
      rs[threadIdx.x] = fmax(rs[threadIdx.x], rs[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = rd[0];
    out[1] = rs[0];
  }
}

// Terminal current spectral density, one block per (contact, energy):
// i_c = Tr[Sigma^<_c G^>_cc - Sigma^>_c G^<_cc] = sum_ab Sigma^<(a,b) G^>(b,a)
// - Sigma^>(a,b) G^<(b,a).  G^r(b,a) and G^<(b,a) come from the stored rows
// (caddr entry (b, a); bit 31: stored as the transposed entry, G^r
// symmetric, G^< anti-Hermitian); G^> = G^< + G^r - G^r+ with G^r+(b,a) =
// conj(G^r(a,b)) = conj(G^r(b,a)).  Block sum in a fixed order.
__global__ void __launch_bounds__(256) k_current(Ctx c, const int32_t* caddr, double* cur) {
  __shared__ double red[256];
  const int cc = blockIdx.x, e = blockIdx.y;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const int nc = sel2(c.nc, cc);
  const int32_t* ca = caddr + (cc ? c.nc[0] * c.nc[0] : 0);
  const double2* S = slab(c, e);
  const double2* sl = sel2(c.sig_l, cc) + (int64_t)(eb + e) * nc * nc;
  const double2* sr = sel2(c.sig_r, cc) + (int64_t)(eb + e) * nc * nc;
  double acc = 0.0;
  for (int q = threadIdx.x; q < nc * nc; q += 256) {
    const int a = q / nc, b = q - a * nc;
    const int32_t code = ca[b * nc + a];
    const int64_t off = code & 0x7fffffff;
    const double2 gr = S[off];
    double2 gl = S[off + c.pdelta];
    if (code < 0) gl = make_double2(-gl.x, gl.y);
    const double2 gg = make_double2(gl.x, gl.y + 2.0 * gr.y);           // G^< + G^r - conj(G^r)
    const double2 s_l = sl[q], s_r = sr[q], s_rt = sr[b * nc + a];
    const double2 s_g = make_double2(s_l.x + s_r.x - s_rt.x, s_l.y + s_r.y + s_rt.y);  // Sigma^>(a,b)
    acc += (s_l.x * gg.x - s_l.y * gg.y) - (s_g.x * gl.x - s_g.y * gl.y);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) cur[(int64_t)(eb + e) * c.ncontacts + cc] = red[0];
}

// Sources of the separate G^> step (Section 2) and of the transmission, per
// (entry, energy of the batch, contact); see launch_form_source.
__global__ void __launch_bounds__(256) k_form_source(Ctx c, double2* src0, double2* src1, int which) {
  const int cc = blockIdx.z, e = blockIdx.y;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const int nc = sel2(c.nc, cc);
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nc * nc) return;
  const int a = q / nc, b = q - a * nc;
  const double2* sr = sel2(c.sig_r, cc) + (int64_t)(eb + e) * nc * nc;
  const double2 r_ab = sr[q], r_ba = sr[b * nc + a];
  double2 v = make_double2(r_ab.x - r_ba.x, r_ab.y + r_ba.y);   // Sigma^r - (Sigma^r)+
  if (which == 0) {
    const double2 l = sel2(c.sig_l, cc)[(int64_t)(eb + e) * nc * nc + q];
    v.x += l.x;
    v.y += l.y;
  } else if (cc == 0) {
    v = make_double2(0.0, 0.0);
  }
  (cc ? src1 : src0)[(int64_t)e * nc * nc + q] = v;
}

__global__ void __launch_bounds__(256) k_epilogue_lesser(Ctx c, double2* out) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int e = blockIdx.y;
  const int eb = ebase(c);
  if (eb + e >= c.nE || q >= c.n) return;
  const SiteDiag sd = c.sdiag[q];
  const double2* S = slab(c, e);
  out[(int64_t)(eb + e) * c.n + q] = S[sd.ol];
}

// T = Tr[Gamma_0 G_01 Gamma_1 G_01+] from X = G (Sigma^r_1 - Sigma^r_1+) G+
// = -i G Gamma_1 G+ held in the G^< fronts: with Gamma_0 = i D_0,
// D_0 = Sigma^r_0 - Sigma^r_0+, T = -Tr[D_0 X_00] = -sum_ab D_0(a,b) X(b,a).
// X is anti-Hermitian like G^<: X(b,a) stored as the transposed entry is
// -conj of it.  One block per energy, a fixed-order block sum.
__global__ void __launch_bounds__(256) k_transmission(Ctx c, const int32_t* caddr, double* T) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  const int eb = ebase(c);
  if (eb + e >= c.nE) return;
  const int nc = c.nc[0];
  const double2* S = slab(c, e);
  const double2* sr = c.sig_r[0] + (int64_t)(eb + e) * nc * nc;
  double acc = 0.0;
  for (int q = threadIdx.x; q < nc * nc; q += 256) {
    const int a = q / nc, b = q - a * nc;
    const int32_t code = caddr[b * nc + a];
    double2 x = S[(int64_t)(code & 0x7fffffff) + c.pdelta];
    if (code < 0) x = make_double2(-x.x, x.y);
    const double2 r_ab = sr[q], r_ba = sr[b * nc + a];
    const double2 d = make_double2(r_ab.x - r_ba.x, r_ab.y + r_ba.y);
    acc -= d.x * x.x - d.y * x.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) T[eb + e] = red[0];
}

void launch_form_source(const Ctx& c, double2* src0, double2* src1, int which, int nb, hipStream_t st) {
  const int m = max(c.nc[0] * c.nc[0], c.ncontacts > 1 ? c.nc[1] * c.nc[1] : 0);
  if (c.ncontacts <= 0 || nb <= 0 || m <= 0) return;
  hipLaunchKernelGGL(k_form_source, dim3((m + 255) / 256, nb, c.ncontacts), dim3(256), 0, st, c, src0, src1,
                     which);
}
void launch_epilogue_lesser(const Ctx& c, int nb, double2* out, hipStream_t st) {
  if (nb > 0) hipLaunchKernelGGL(k_epilogue_lesser, dim3((c.n + 255) / 256, nb), dim3(256), 0, st, c, out);
}
void launch_transmission(const Ctx& c, const int32_t* caddr, int nb, double* T, hipStream_t st) {
  if (nb > 0 && c.ncontacts >= 2) hipLaunchKernelGGL(k_transmission, dim3(nb), dim3(256), 0, st, c, caddr, T);
}

void launch_current(const Ctx& c, const int32_t* caddr, int nb, double* cur, hipStream_t st) {
  if (c.ncontacts <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_current, dim3(c.ncontacts, nb), dim3(256), 0, st, c, caddr, cur);
}

void launch_scba_mix(const double2* dgr, const double2* dgl, double2* sr, double2* sl, int64_t count,
                     double d0, double mix, double* part, double* out, hipStream_t st) {
  const int nblk = (int)std::min<int64_t>(kScbaBlocks, std::max<int64_t>(1, (count + 255) / 256));
  hipLaunchKernelGGL(k_scba_mix, dim3(nblk), dim3(256), 0, st, dgr, dgl, sr, sl, count, d0, mix, part);
  hipLaunchKernelGGL(k_scba_max, dim3(1), dim3(256), 0, st, part, nblk, out);
}

void launch_anc_g(const Ctx& c, const ScatCtx& x, const ColItem* it, int nit, int nb, int tile_rows,
                  bool leaves, hipStream_t st) {
  if (nit <= 0) return;
  const dim3 grid(nit, nb), blk(256);
  if (leaves) {
    if (tile_rows <= 16) hipLaunchKernelGGL((k_anc_g_leaf<16, 7>), grid, blk, 0, st, c, x, it);
    else if (tile_rows <= 32) hipLaunchKernelGGL((k_anc_g_leaf<32, 4>), grid, blk, 0, st, c, x, it);
    else hipLaunchKernelGGL((k_anc_g_leaf<64, 3>), grid, blk, 0, st, c, x, it);
  } else {
    if (tile_rows <= 16) hipLaunchKernelGGL(k_anc_g<16>, grid, blk, 0, st, c, x, it);
    else if (tile_rows <= 32) hipLaunchKernelGGL(k_anc_g<32>, grid, blk, 0, st, c, x, it);
    else hipLaunchKernelGGL(k_anc_g<64>, grid, blk, 0, st, c, x, it);
  }
}

void launch_anc_n(const Ctx& c, const ScatCtx& x, const ColItem* it, int nit, int nb, int tile_rows,
                  hipStream_t st) {
  if (nit <= 0) return;
  if (tile_rows <= 16) hipLaunchKernelGGL(k_anc_n<16>, dim3(nit, nb), dim3(256), 0, st, c, x, it);
  else if (tile_rows <= 32) hipLaunchKernelGGL(k_anc_n<32>, dim3(nit, nb), dim3(256), 0, st, c, x, it);
  else hipLaunchKernelGGL(k_anc_n<64>, dim3(nit, nb), dim3(256), 0, st, c, x, it);
}

void launch_anc_p0(const Ctx& c, const ScatCtx& x, const int32_t* cls, int ncl, int nb, int tile_rows,
                   hipStream_t st) {
  if (ncl <= 0) return;
  if (tile_rows <= 16) hipLaunchKernelGGL(k_anc_p0<16>, dim3(ncl, nb), dim3(256), 0, st, c, x, cls);
  else if (tile_rows <= 32) hipLaunchKernelGGL(k_anc_p0<32>, dim3(ncl, nb), dim3(256), 0, st, c, x, cls);
  else hipLaunchKernelGGL(k_anc_p0<64>, dim3(ncl, nb), dim3(256), 0, st, c, x, cls);
}

}  // namespace ndg
