// Device helpers shared by the kernel files: complex tiles on the FP64
// matrix cores, fault reporting, workspace addressing.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ndg {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int KC = 16;  // K chunk staged in LDS per step

// A staged for R rows (R >= the tile's TM: smaller tiles take less LDS, so
// more blocks fit on a CU), B for 64 columns
template <int R>
struct GemmSmemR {
  double ar[R][KC + 1], ai[R][KC + 1];
  double br[KC][64 + 1], bi[KC][64 + 1];
};
using GemmSmem = GemmSmemR<64>;

struct ZTile {
  v4d re[2][2];
  v4d im[2][2];
};

__device__ inline void ztile_zero(ZTile& a) {
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      a.re[m][n] = v4d{0, 0, 0, 0};
      a.im[m][n] = v4d{0, 0, 0, 0};
    }
}

__device__ inline double2 cz() { return make_double2(0.0, 0.0); }

// Element cc (0 or 1) of a per-contact pair without dynamic indexing (which
// would move the enclosing struct to scratch memory).
template <class T>
__device__ inline T sel2(const T (&a)[2], int cc) { return cc ? a[1] : a[0]; }
__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc += p x as four FMAs
__device__ inline void cmac(double2& acc, double2 p, double2 x) {
  acc.x = fma(p.x, x.x, acc.x);
  acc.x = fma(-p.y, x.y, acc.x);
  acc.y = fma(p.x, x.y, acc.y);
  acc.y = fma(p.y, x.x, acc.y);
}

// Tile shapes: a 256-thread block computes a TM x 64 complex tile, TM in
// {64, 32, 16} (TM follows the cluster size so small clusters do not fill
// matrix-core tiles with padding).  Waves: 2 x 2 of 32 x 32 for TM = 64,
// 1 x 4 of TM x 16 otherwise.
template <int TM>
struct TileShape {
  static constexpr int WM = TM == 64 ? 2 : 1;        // waves along M
  static constexpr int WN = 4 / WM;                  // waves along N
  static constexpr int MB = TM / WM / 16;            // 16-row blocks per wave
  static constexpr int NB = 64 / WN / 16;            // 16-column blocks per wave
};

// The matrix-core work on one staged chunk: the 4-deep steps below kend, on
// this wave's 16 x 16 blocks of the tile (at rows wr, columns wc); with PRED
// the blocks wholly outside the first live_m rows and live_n columns are
// skipped (a choice uniform over the wave).
template <int TM, bool PRED, bool RAGGED, int R>
__device__ __forceinline__ void mma_chunk(const GemmSmemR<R>& sm, ZTile& acc, int wr, int wc, int lane, int kend,
                                          int live_m, int live_n) {
  using T = TileShape<TM>;
#pragma unroll
  for (int k4 = 0; k4 < KC; k4 += 4) {
    if (RAGGED && k4 >= kend) break;
    const int kq = k4 + (lane >> 4);
    double are[T::MB], aim[T::MB], bre[T::NB], bim[T::NB];
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
        if (PRED && (wr + 16 * m >= live_m || wc + 16 * n >= live_n)) continue;
        acc.re[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[m], bre[n], acc.re[m][n], 0, 0, 0);
        acc.re[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(-aim[m], bim[n], acc.re[m][n], 0, 0, 0);
        acc.im[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(are[m], bim[n], acc.im[m][n], 0, 0, 0);
        acc.im[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim[m], bre[n], acc.im[m][n], 0, 0, 0);
      }
  }
}

// acc += A (TM x K) * B (K x 64).  fa(i, k) and fb(k, j) return the complex
// operand (and 0 outside the live range); A_IFAST / B_KFAST select which index
// runs fastest across threads while staging, to match the memory layout.
// Every thread of the 256-thread block must call this.
// With PF, the operands of chunk k0 + KC are loaded into registers while the
// matrix cores work on chunk k0 (the global-load latency hides behind the
// MFMAs); kernels that inline several products turn it off to stay within
// the register file.  With RAGGED the last chunk runs only the 4-deep MFMA
// steps that hold live K (products with short K, where a full 16-deep chunk
// would mostly multiply zeros).  Only the first live_m rows and live_n
// columns of the tile are live (fa and fb return 0 beyond them): in tiles of
// fewer than 64 rows a wave skips the matrix-core work of its 16 x 16 blocks
// that lie wholly outside (a ragged edge, or a block narrower than the tile;
// the 64-row tiles keep one code path, within their register budget).
template <int TM, bool A_IFAST, bool B_KFAST, bool PF = true, int R = 64, bool RAGGED = false, class FA,
          class FB>
__device__ void zgemm_acc_t(int K, FA fa, FB fb, ZTile& acc, GemmSmemR<R>& sm, int live_m = TM, int live_n = 64) {
  static_assert(R >= TM, "staging rows");
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
  const bool all_live = wr + 16 * T::MB <= live_m && wc + 16 * T::NB <= live_n;
  // staging index of operand element q of this thread
  auto a_idx = [&](int q, int& i, int& kk) {
    const int idx = t + 256 * q;
    if (A_IFAST) { i = idx % TM; kk = idx / TM; }
    else { kk = idx & (KC - 1); i = idx / KC; }
  };
  auto b_idx = [&](int q, int& kk, int& j) {
    const int idx = t + 256 * q;
    if (B_KFAST) { kk = idx & (KC - 1); j = idx / KC; }
    else { j = idx & 63; kk = idx >> 6; }
  };
  double2 pa[PF ? TM / 16 : 1], pb[PF ? 4 : 1];
  auto load = [&](int k0) {
    if constexpr (PF) {
#pragma unroll
      for (int q = 0; q < TM / 16; ++q) {
        int i, kk;
        a_idx(q, i, kk);
        pa[q] = (k0 + kk < K) ? fa(i, k0 + kk) : cz();
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int kk, j;
        b_idx(q, kk, j);
        pb[q] = (k0 + kk < K) ? fb(k0 + kk, j) : cz();
      }
    }
  };
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int q = 0; q < TM / 16; ++q) {
      int i, kk;
      a_idx(q, i, kk);
      double2 v;
      if constexpr (PF) v = pa[q];
      else v = (k0 + kk < K) ? fa(i, k0 + kk) : cz();
      sm.ar[i][kk] = v.x;
      sm.ai[i][kk] = v.y;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int kk, j;
      b_idx(q, kk, j);
      double2 v;
      if constexpr (PF) v = pb[q];
      else v = (k0 + kk < K) ? fb(k0 + kk, j) : cz();
      sm.br[kk][j] = v.x;
      sm.bi[kk][j] = v.y;
    }
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
    const int kend = RAGGED ? min(KC, K - k0) : KC;
    if (TM == 64 || all_live) mma_chunk<TM, false, RAGGED>(sm, acc, wr, wc, lane, kend, live_m, live_n);
    else mma_chunk<TM, true, RAGGED>(sm, acc, wr, wc, lane, kend, live_m, live_n);
    __syncthreads();
  }
}

// acc += A (TM x K) * B (K x 64) with B gathered through an index table:
// fidx(k, j) loads the table entry of B(k, j), fval(entry, j) the value it
// points to (0 for columns outside the tile).  The table entries run one chunk ahead of the values: while the
// matrix cores work on chunk k0, the values of chunk k0 + KC (whose entries
// arrived during the previous chunk) and the entries of chunk k0 + 2 KC are
// in flight, so each chunk waits for one memory round trip instead of two
// dependent ones.  A is read as in zgemm_acc_t (A_IFAST), B with j fastest;
// live_m and live_n as there.
template <int TM, bool A_IFAST, int R, class FA, class FI, class FV>
__device__ void zgemm_acc_gather_t(int K, FA fa, FI fidx, FV fval, ZTile& acc, GemmSmemR<R>& sm, int live_m = TM,
                                   int live_n = 64) {
  static_assert(R >= TM, "staging rows");
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
  const bool all_live = wr + 16 * T::MB <= live_m && wc + 16 * T::NB <= live_n;
  auto a_idx = [&](int q, int& i, int& kk) {
    const int idx = t + 256 * q;
    if (A_IFAST) { i = idx % TM; kk = idx / TM; }
    else { kk = idx & (KC - 1); i = idx / KC; }
  };
  const int bj = t & 63, bk = t >> 6;  // B element q of this thread: (bk + 4q, bj)
  double2 pa[TM / 16], pb[4];
  int32_t pm[4];
  auto load_a = [&](int k0) {
#pragma unroll
    for (int q = 0; q < TM / 16; ++q) {
      int i, kk;
      a_idx(q, i, kk);
      pa[q] = (k0 + kk < K) ? fa(i, k0 + kk) : cz();
    }
  };
  auto load_idx = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) pm[q] = (k0 + bk + 4 * q < K) ? fidx(k0 + bk + 4 * q, bj) : 0;
  };
  auto load_val = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) pb[q] = (k0 + bk + 4 * q < K) ? fval(pm[q], bj) : cz();
  };
  if (K > 0) {
    load_a(0);
    load_idx(0);
    load_val(0);
    load_idx(KC);
  }
  for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int q = 0; q < TM / 16; ++q) {
      int i, kk;
      a_idx(q, i, kk);
      sm.ar[i][kk] = pa[q].x;
      sm.ai[i][kk] = pa[q].y;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sm.br[bk + 4 * q][bj] = pb[q].x;
      sm.bi[bk + 4 * q][bj] = pb[q].y;
    }
    __syncthreads();
    if (k0 + KC < K) {
      load_a(k0 + KC);
      load_val(k0 + KC);
      load_idx(k0 + 2 * KC);
    }
    if (TM == 64 || all_live) mma_chunk<TM, false, false>(sm, acc, wr, wc, lane, KC, live_m, live_n);
    else mma_chunk<TM, true, false>(sm, acc, wr, wc, lane, KC, live_m, live_n);
    __syncthreads();
  }
}

template <bool A_IFAST, bool B_KFAST, class FA, class FB>
__device__ void zgemm_acc(int K, FA fa, FB fb, ZTile& acc, GemmSmem& sm, int live_m = 64, int live_n = 64) {
  zgemm_acc_t<64, A_IFAST, B_KFAST, true>(K, fa, fb, acc, sm, live_m, live_n);
}

// Calls fs(i, j, re, im) for every tile element this thread holds
// (v_mfma_f64_16x16x4: lane l, register r -> row l/16 + 4r, column l%16).
template <int TM, class FS>
__device__ inline void ztile_store_t(const ZTile& acc, FS fs) {
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
#pragma unroll
  for (int m = 0; m < T::MB; ++m)
#pragma unroll
    for (int n = 0; n < T::NB; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr + m * 16 + (lane >> 4) + 4 * r;
        const int j = wc + n * 16 + (lane & 15);
        fs(i, j, acc.re[m][n][r], acc.im[m][n][r]);
      }
}

template <class FS>
__device__ inline void ztile_store(const ZTile& acc, FS fs) {
  ztile_store_t<64>(acc, fs);
}

// ztile_store_t of acc + fl(i, j): every fl load of this thread is issued
// before the first store (stores may alias the loads, so a load after a
// store would wait for it), then fs(i, j, re, im) with the sums.
// With BY_ROW the loads and stores go one 16-row block at a time (half the
// registers for the loaded values, two rounds of loads).
template <int TM, bool BY_ROW = false, class FL, class FS>
__device__ inline void ztile_store_add_t(const ZTile& acc, FL fl, FS fs) {
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
  constexpr int G = BY_ROW ? 1 : T::MB;  // row blocks per round
#pragma unroll
  for (int m0 = 0; m0 < T::MB; m0 += G) {
    double2 add[G][T::NB][4];
#pragma unroll
    for (int m = 0; m < G; ++m)
#pragma unroll
      for (int n = 0; n < T::NB; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          add[m][n][r] = fl(wr + (m0 + m) * 16 + (lane >> 4) + 4 * r, wc + n * 16 + (lane & 15));
#pragma unroll
    for (int m = 0; m < G; ++m)
#pragma unroll
      for (int n = 0; n < T::NB; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          fs(wr + (m0 + m) * 16 + (lane >> 4) + 4 * r, wc + n * 16 + (lane & 15),
             acc.re[m0 + m][n][r] + add[m][n][r].x, acc.im[m0 + m][n][r] + add[m][n][r].y);
  }
}

// Calls fs(i, j, re, im) with references to every tile element this thread
// holds (same layout as ztile_store_t), to update the tile in place.
template <int TM, class FS>
__device__ inline void ztile_apply_t(ZTile& acc, FS fs) {
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
#pragma unroll
  for (int m = 0; m < T::MB; ++m)
#pragma unroll
    for (int n = 0; n < T::NB; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr + m * 16 + (lane >> 4) + 4 * r;
        const int j = wc + n * 16 + (lane & 15);
        double re = acc.re[m][n][r], im = acc.im[m][n][r];
        fs(i, j, re, im);
        acc.re[m][n][r] = re;
        acc.im[m][n][r] = im;
      }
}


// ---------------------------------------------------------------------------
// Complex FP32 tiles on the FP32 matrix cores (mixed-precision path):
// v_mfma_f32_16x16x4_f32 with FP32 accumulation; operands are read in FP64
// and rounded to FP32 while staging.  Output layout: lane l, register r ->
// row 4 (l / 16) + r, column l % 16.
typedef float v4f __attribute__((ext_vector_type(4)));

template <int R>
struct GemmSmem32R {
  float ar[R][KC + 1], ai[R][KC + 1];
  float br[KC][64 + 1], bi[KC][64 + 1];
};
using GemmSmem32 = GemmSmem32R<64>;

struct ZTile32 {
  v4f re[2][2];
  v4f im[2][2];
};

__device__ inline void ztile32_zero(ZTile32& a) {
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      a.re[m][n] = v4f{0, 0, 0, 0};
      a.im[m][n] = v4f{0, 0, 0, 0};
    }
}

template <int TM, bool A_IFAST, bool B_KFAST, int R = 64, class FA, class FB>
__device__ void zgemm32_acc_t(int K, FA fa, FB fb, ZTile32& acc, GemmSmem32R<R>& sm) {
  static_assert(R >= TM, "staging rows");
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
  double2 pa[TM / 16], pb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < TM / 16; ++q) {
      const int idx = t + 256 * q;
      int i, kk;
      if (A_IFAST) { i = idx % TM; kk = idx / TM; }
      else { kk = idx & (KC - 1); i = idx / KC; }
      pa[q] = (k0 + kk < K) ? fa(i, k0 + kk) : cz();
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = t + 256 * q;
      int kk, j;
      if (B_KFAST) { kk = idx & (KC - 1); j = idx / KC; }
      else { j = idx & 63; kk = idx >> 6; }
      pb[q] = (k0 + kk < K) ? fb(k0 + kk, j) : cz();
    }
  };
  if (K > 0) load(0);
  for (int k0 = 0; k0 < K; k0 += KC) {
#pragma unroll
    for (int q = 0; q < TM / 16; ++q) {
      const int idx = t + 256 * q;
      int i, kk;
      if (A_IFAST) { i = idx % TM; kk = idx / TM; }
      else { kk = idx & (KC - 1); i = idx / KC; }
      sm.ar[i][kk] = (float)pa[q].x;
      sm.ai[i][kk] = (float)pa[q].y;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = t + 256 * q;
      int kk, j;
      if (B_KFAST) { kk = idx & (KC - 1); j = idx / KC; }
      else { j = idx & 63; kk = idx >> 6; }
      sm.br[kk][j] = (float)pb[q].x;
      sm.bi[kk][j] = (float)pb[q].y;
    }
    __syncthreads();
    if (k0 + KC < K) load(k0 + KC);
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      const int kq = k4 + (lane >> 4);
      float are[2], aim[2], bre[2], bim[2];
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
          acc.re[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[m], bre[n], acc.re[m][n], 0, 0, 0);
          acc.re[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(-aim[m], bim[n], acc.re[m][n], 0, 0, 0);
          acc.im[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[m], bim[n], acc.im[m][n], 0, 0, 0);
          acc.im[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[m], bre[n], acc.im[m][n], 0, 0, 0);
        }
    }
    __syncthreads();
  }
}

template <int TM, class FS>
__device__ inline void ztile32_store_t(const ZTile32& acc, FS fs) {
  using T = TileShape<TM>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = (w / T::WN) * (TM / T::WM), wc = (w % T::WN) * (64 / T::WN);
#pragma unroll
  for (int m = 0; m < T::MB; ++m)
#pragma unroll
    for (int n = 0; n < T::NB; ++n)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr + m * 16 + 4 * (lane >> 4) + r;
        const int j = wc + n * 16 + (lane & 15);
        fs(i, j, (double)acc.re[m][n][r], (double)acc.im[m][n][r]);
      }
}

// Precision-generic front ends: P64 = true selects the FP64 tiles.
template <bool P64>
struct Gemm;
template <>
struct Gemm<true> {
  using Tile = ZTile;
  using Smem = GemmSmem;
  template <int R>
  using SmemT = GemmSmemR<R>;
  __device__ static void zero(Tile& a) { ztile_zero(a); }
  template <int TM, bool AI, bool BK, bool PF = true, int R, class FA, class FB>
  __device__ static void acc(int K, FA fa, FB fb, Tile& t, SmemT<R>& sm, int live_m = TM, int live_n = 64) {
    zgemm_acc_t<TM, AI, BK, PF>(K, fa, fb, t, sm, live_m, live_n);
  }
  template <int TM, class FS>
  __device__ static void store(const Tile& t, FS fs) { ztile_store_t<TM>(t, fs); }
};
template <>
struct Gemm<false> {
  using Tile = ZTile32;
  using Smem = GemmSmem32;
  template <int R>
  using SmemT = GemmSmem32R<R>;
  __device__ static void zero(Tile& a) { ztile32_zero(a); }
  template <int TM, bool AI, bool BK, bool PF = true, int R, class FA, class FB>
  __device__ static void acc(int K, FA fa, FB fb, Tile& t, SmemT<R>& sm, int = TM, int = 64) {
    zgemm32_acc_t<TM, AI, BK>(K, fa, fb, t, sm);
  }
  template <int TM, class FS>
  __device__ static void store(const Tile& t, FS fs) { ztile32_store_t<TM>(t, fs); }
};

// ---------------------------------------------------------------------------
// Gauss-Jordan elimination with partial pivoting on a matrix held in
// registers: thread (jt, i0) = (t % JS, t / JS) owns rows i0 + RS*m and
// columns jt + JS*q.  Pivots are taken in place (no row interchanges): step
// k sweeps column k with the largest unused row p_k among the first s rows,
// so after s steps the entry in storage row p_k, column c < s is
// (A^{-1})[k][p_c], rows and columns >= s keep their meaning, and
//     [[A_ii, A_iB], [A_Bi, A_BB]]  ->  [[A_ii^{-1} (permuted), A_ii^{-1} A_iB (rows permuted)],
//                                        [-A_Bi A_ii^{-1},      A_BB - A_Bi A_ii^{-1} A_iB]].
// ---------------------------------------------------------------------------
// Maximum of a 32-bit key over the 64 lanes of a wavefront, returned to
// every lane: a butterfly inside each row of 16 lanes through DPP (quad
// permutations, then row rotations by 4 and 8), then the four row maxima
// read as scalars.
__device__ inline unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));  // row_ror 4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));  // row_ror 8
  const unsigned r0 = (unsigned)__builtin_amdgcn_readlane((int)v, 0);
  const unsigned r1 = (unsigned)__builtin_amdgcn_readlane((int)v, 16);
  const unsigned r2 = (unsigned)__builtin_amdgcn_readlane((int)v, 32);
  const unsigned r3 = (unsigned)__builtin_amdgcn_readlane((int)v, 48);
  return max(max(r0, r1), max(r2, r3));
}

// 1 / x for x > 0: the hardware estimate refined by two Newton-Raphson steps
// r <- r (2 - x r) (each doubles the number of correct bits).
__device__ inline double recip_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

__device__ inline double lane_read(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int SF, int NT, int JS>
struct RegGJ {
  static constexpr int RS = NT / JS;
  static constexpr int NR = (SF + RS - 1) / RS;
  static constexpr int NC = (SF + JS - 1) / JS;
  static_assert(NT % JS == 0, "thread grid");
  // one wavefront searches the pivot rows: a row per lane, two above 64
  static_assert(SF <= 128, "pivot rows are searched by one wavefront");
  static constexpr bool kTwo = SF > 64;
  static_assert(NT % 64 == 0, "whole wavefronts");
  struct Smem {
    double2 col[2][NR * RS];
    double2 row[2][NC * JS];
    int piv[SF], pinv[SF];
  };
  double re[NR][NC], im[NR][NC];
  int jt, i0;

  __device__ RegGJ(int t) : jt(t % JS), i0(t / JS) {}
  __device__ int row(int m) const { return i0 + RS * m; }
  __device__ int col(int q) const { return jt + JS * q; }

  // s pivot steps; returns false if a pivot was exactly zero.  Per step:
  // the owners of column k publish it and clear it (its new value is
  // -M[i][k] d); after a barrier every wavefront finds the pivot row p by a
  // wave-wide maximum of packed (magnitude, row) keys and the owners of row
  // p publish it; after a second barrier every thread applies
  // M[i][j] -= M[i][k] x_j (x_j = M[p][j] d, x_k = d) to its whole tile
  // and the owners of row p then overwrite it with x.  The steps run in
  // groups of JS (one register column q_k per group, unrolled), so the
  // pivot column's register index is a constant; the pivot row's register
  // slot m_p = p / RS is uniform over the block, and with several columns
  // per thread the row is published from a branch per slot rather than
  // through selects over all slots.
  __device__ bool run(Smem& sm, int s) {
    const int t = i0 * JS + jt, lane = t & 63;
    unsigned long long used = 0, used_hi = 0;  // rows 0..63, 64..127 already pivots
    bool ok = true;
#pragma unroll
    for (int qk = 0; qk < NC; ++qk) {
      for (int kj = 0; kj < JS; ++kj) {
        const int k = qk * JS + kj;
        if (k >= s) break;
        const int buf = k & 1;
        if (jt == kj) {
#pragma unroll
          for (int m = 0; m < NR; ++m) {
            sm.col[buf][row(m)] = make_double2(re[m][qk], im[m][qk]);
            re[m][qk] = 0.0;
            im[m][qk] = 0.0;
          }
        }
        __syncthreads();
        // key = valid bit | magnitude |Re| + |Im| as a float (its bits
        // order like the values; 16 mantissa bits kept) | (63 - row): the
        // largest magnitude wins, near-ties go to the lower row; every
        // unused row below s has the valid bit, so p is always a valid row
        // (a NaN column picks a NaN row)
        const double2 v = lane < s ? sm.col[buf][lane] : make_double2(0.0, 0.0);
        unsigned key = 0;
        int p;
        double2 a;
        if constexpr (!kTwo) {
          if (lane < s && !((used >> lane) & 1ull)) {
            const float mg = (float)(fabs(v.x) + fabs(v.y));
            key = 0x80000000u | ((__float_as_uint(mg) >> 1) & 0x7FFFFFC0u) | (unsigned)(63 - lane);
          }
          key = wave_max_u32(key);
          p = 63 - (int)(key & 63u);
          a = make_double2(lane_read(v.x, p), lane_read(v.y, p));
        } else {
          // rows lane and lane + 64; 7 row bits, (127 - row) so near-ties go
          // to the lower row
          const double2 v2 = lane + 64 < s ? sm.col[buf][lane + 64] : make_double2(0.0, 0.0);
          if (lane < s && !((used >> lane) & 1ull)) {
            const float mg = (float)(fabs(v.x) + fabs(v.y));
            key = 0x80000000u | ((__float_as_uint(mg) >> 1) & 0x7FFFFF80u) | (unsigned)(127 - lane);
          }
          if (lane + 64 < s && !((used_hi >> lane) & 1ull)) {
            const float mg = (float)(fabs(v2.x) + fabs(v2.y));
            const unsigned k2 = 0x80000000u | ((__float_as_uint(mg) >> 1) & 0x7FFFFF80u) | (unsigned)(63 - lane);
            key = k2 > key ? k2 : key;
          }
          key = wave_max_u32(key);
          p = 127 - (int)(key & 127u);
          const double2 w = p < 64 ? v : v2;
          a = make_double2(lane_read(w.x, p & 63), lane_read(w.y, p & 63));
        }
        const int mp = p / RS;
        const bool own_p = i0 == p % RS;
        if constexpr (NC > 1) {
#pragma unroll
          for (int m = 0; m < NR; ++m) {
            if (m == mp) {
              // distinct per slot, so the branches are not merged into selects
              asm volatile("; pivot row slot %0" ::"i"(m));
              if (own_p) {
#pragma unroll
                for (int q = 0; q < NC; ++q) sm.row[buf][col(q)] = make_double2(re[m][q], im[m][q]);
              }
            }
          }
        } else if (own_p) {
          double vr = 0.0, vi = 0.0;
#pragma unroll
          for (int m = 0; m < NR; ++m)
            if (m == mp) {
              vr = re[m][0];
              vi = im[m][0];
            }
          sm.row[buf][col(0)] = make_double2(vr, vi);
        }
        if (t == 0) {
          sm.piv[k] = p;
          sm.pinv[p] = k;
        }
        if (p < 64) used |= 1ull << p;
        else used_hi |= 1ull << (p - 64);
        const double den = a.x * a.x + a.y * a.y;
        double dr = 0.0, di = 0.0;
        if (den > 0.0) {
          const double r = recip_pos(den);
          dr = a.x * r;
          di = -a.y * r;
        } else {
          ok = false;
        }
        __syncthreads();
        double2 ck[NR], pr[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) pr[q] = sm.row[buf][col(q)];
#pragma unroll
        for (int m = 0; m < NR; ++m) ck[m] = sm.col[buf][row(m)];
        double xr[NC], xi[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          xr[q] = fma(pr[q].x, dr, -pr[q].y * di);
          xi[q] = fma(pr[q].x, di, pr[q].y * dr);
          if (q == qk) {
            xr[q] = jt == kj ? dr : xr[q];
            xi[q] = jt == kj ? di : xi[q];
          }
#pragma unroll
          for (int m = 0; m < NR; ++m) {
            re[m][q] = fma(-ck[m].x, xr[q], re[m][q]);
            re[m][q] = fma(ck[m].y, xi[q], re[m][q]);
            im[m][q] = fma(-ck[m].x, xi[q], im[m][q]);
            im[m][q] = fma(-ck[m].y, xr[q], im[m][q]);
          }
        }
        if (own_p) {
#pragma unroll
          for (int m = 0; m < NR; ++m)
            if (m == mp) {
#pragma unroll
              for (int q = 0; q < NC; ++q) {
                re[m][q] = xr[q];
                im[m][q] = xi[q];
              }
            }
        }
      }
    }
    __syncthreads();  // piv / pinv complete
    return ok;
  }
};

__device__ inline void raise_fault(int32_t* status, int code, int e, int cl) {
  if (atomicCAS(status, 0, code) == 0) {
    atomicExch(status + 1, e);
    atomicExch(status + 2, cl);
  }
}

__device__ inline double2* slab(const Ctx& c, int e) { return c.ws + (int64_t)e * c.stride; }

// Entry (u, v) of X_{B,B} for a cluster with boundary B (X = G^r, or G^<
// when lesser): read from the stored rows of the lower owning cluster, using
// G^r_{yx} = G^r_{xy} and G^<_{yx} = -conj(G^<_{xy}) for the other order.
// The table entry (offset in the energy's slab, sign bit set when the entry
// is read in the other order) and the value it points to.
__device__ inline int32_t gather_bb_entry(const Ctx& c, const ClusterDesc& d, int u, int v) {
  return c.gaddr[d.o_gaddr + (int64_t)u * d.b + v];
}
__device__ inline double2 gather_bb_value(const Ctx& c, const double2* S, int32_t m, bool lesser) {
  const double2 x = S[(int64_t)(m & 0x7FFFFFFF) + (lesser ? c.pdelta : 0)];
  return (m < 0 && lesser) ? make_double2(-x.x, x.y) : x;
}
__device__ inline double2 gather_bb(const Ctx& c, const double2* S, const ClusterDesc& d, int u,
                                    int v, bool lesser) {
  return gather_bb_value(c, S, gather_bb_entry(c, d, u, v), lesser);
}

// Entry (u, v) of X_{B,B} where B is a run of one ancestor's points
// (ClusterDesc::o_bbd): a dense block of that ancestor's stored rows, no
// lookup.
__device__ inline double2 direct_bb(const Ctx& c, const double2* S, const ClusterDesc& d, int u, int v,
                                    bool lesser) {
  return S[d.o_bbd + (int64_t)u * d.bbd_ld + v + (lesser ? c.pdelta : 0)];
}

// The exact X_ii block of G^r is complex symmetric and that of G^< anti-
// Hermitian; the extraction computes it as A_ii^{-1} + Psi_i X_{B,i}, whose
// two triangles carry different rounding, amplified by large Psi.  Replacing
// the stored block by its symmetric (anti-Hermitian) part before any
// descendant gathers from it keeps that error out of the descendants: a
// descendant reading either triangle then sees the same value.  In place on
// the s x s block (row stride f) after the whole block is written: one
// thread per pair (r, c >= r), every block thread taking part.
__device__ inline void symmetrize_block(double2* X, int s, int f, bool lesser) {
  __threadfence_block();
  __syncthreads();
  for (int q = threadIdx.x; q < s * s; q += blockDim.x) {
    const int r = q / s, cc = q - r * s;
    if (cc < r) continue;
    const double2 a = X[(int64_t)r * f + cc], b = X[(int64_t)cc * f + r];
    if (lesser) {
      // (a - conj(b)) / 2 at (r, c), its negated conjugate at (c, r)
      const double2 m = make_double2(0.5 * (a.x - b.x), 0.5 * (a.y + b.y));
      X[(int64_t)r * f + cc] = m;
      X[(int64_t)cc * f + r] = make_double2(-m.x, m.y);
    } else {
      const double2 m = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y + b.y));
      X[(int64_t)r * f + cc] = m;
      X[(int64_t)cc * f + r] = m;
    }
  }
}

// First energy of the batch this launch processes.
__device__ inline int ebase(const Ctx& c) { return c.e0p ? c.e0 + *c.e0p : c.e0; }

// Workgroup -> (item, energy) of a grid (items, energies).  The dispatcher
// deals workgroups to the eight XCDs round-robin by linear index, and each
// XCD has its own L2.  Here every XCD takes every eighth energy and runs its
// energies in groups of eight, item by item: the column tiles of one cluster
// at one energy (which read the two triangles of the same symmetric block)
// and one cluster's address tables over eight energies then meet in the same
// L2 close together in time.  A bijection of the grid; the plain order when
// the energy count is not a multiple of 8.
struct WorkIdx {
  int item, e;
};
__device__ inline WorkIdx xcd_work() {
  const int nit = gridDim.x, nb = gridDim.y;
  if (nb & 7) return {(int)blockIdx.x, (int)blockIdx.y};
  const int lin = blockIdx.x + blockIdx.y * nit;
  const int xcd = lin & 7, m = lin >> 3, per = nb >> 3;
  const int g = (per & 7) ? 1 : 8;
  const int grp = m / (nit * g), r = m - grp * nit * g;
  return {r / g, ((grp * g + r % g) << 3) + xcd};
}

}  // namespace ndg
