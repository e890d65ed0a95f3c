// Dense complex linear algebra on CDNA4 matrix cores (MFMA 16x16x4, FP64 and FP32).
//
// * zgemm:        batched C = alpha op(A) op(B) + beta C, op in {N, conjugate-transpose},
//                 64x64 output tiles, 256 threads, optional lower-triangular tile grid
//                 (Hermitian rank-k updates) and split-K with a deterministic reduction.
// * potrf_diag:   Cholesky of one 64x64 diagonal block per matrix in LDS, plus the
//                 explicit inverse of the factor (used to turn panel and block
//                 triangular solves into GEMMs).
//
// Complex products in the tiled GEMM take three real MFMA products (Karatsuba), those
// of the streaming kernels four (FP64) or three (FP32).  The MFMA is fed the
// B tile as its first operand and the A tile as its second, so the 16x16 result
// it returns is C transposed: each lane then holds four *columns* of one row,
// and lanes 0..15 cover 16 consecutive rows, which makes the stores to
// column-major C contiguous.
#include <hip/hip_ext.h>

#include "phx_common.h"
#include "phx_internal.h"

namespace phx {

// One workgroup (4 waves) computes a BM x BN tile of C; wave w covers rows
// (w % WM) * 32 .. +32 and columns (w / WM) * 32 .. +32 with 2 x 2 MFMA blocks.
// Shapes: 64 x 64 (WM = 2) for square work, 128 x 32 (WM = 4) for the narrow
// right-hand-side blocks of the triangular solves and subspace updates.
// MODE: 0 general, 1 lower-triangular tile grid (Hermitian rank-k update).
template <typename R, int OPA, int OPB, int BM, int BN, int MODE>
__global__ __launch_bounds__(256, 3) void zgemm_kernel(GemmArgs<R> g) {
  typedef C_t<R> C;
  typedef typename acc_t<R>::type ACC;
  constexpr int WM = BM / 32;
  static_assert(WM * (BN / 32) == 4, "four waves per tile");
  // KS: depth of the LDS stage (16 for FP32, 8 for FP64: the same bytes).
  constexpr int KS = sizeof(R) == 4 ? 16 : 8;
  // per-thread staging: A holds BM*KS elements, B holds KS*BN, in groups of VA / VB
  // consecutive elements along the operand's contiguous dimension
  constexpr int NA = BM * KS / 256, NB = BN * KS / 256;
  constexpr int VA = NA < 4 ? NA : 4, VB = NB < 4 ? NB : 4;
  constexpr int GA = NA / VA, GB = NB / VB;
  __shared__ R Asr[KS][BM + 4], Asi[KS][BM + 4], Bsr[KS][BN + 4], Bsi[KS][BN + 4];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WM, wc = wave / WM;
  // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin by linear id, so
  // the linear ids are remapped to give every XCD one contiguous range of
  // (tile, batch) indices; neighbouring tiles share operand panels in that XCD's L2.
  long tile_lin, bat;
  {
    const long nx = gridDim.x, total = nx * (long)gridDim.y;
    const long lin = blockIdx.x + nx * (long)blockIdx.y;
    const long per = total / 8, rem = total % 8, xcd = lin % 8, idx = lin / 8;
    const long logical = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
    tile_lin = logical % nx;
    bat = logical / nx;
  }
  int ti, tj;
  if (MODE == 1) {
    const long t = tile_lin;
    long r = (long)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    ti = (int)r;
    tj = (int)(t - r * (r + 1) / 2);
  } else {
    const int tm = (g.M + BM - 1) / BM;
    ti = (int)(tile_lin % tm);
    tj = (int)(tile_lin / tm);
  }
  const int row0 = ti * BM, col0 = tj * BN;
  const int b = g.bidx ? g.bidx[bat / g.kdiv] * g.kdiv + (int)(bat % g.kdiv) : (int)bat;
  if (g.kact && !g.kact[b / g.kdiv]) return;  // whole workgroup: a converged k-point
  const int sp = blockIdx.z;
  const C* A = g.A + (long)(g.amap ? g.amap[b] : b / g.dA) * g.sA;
  const C* B = g.B + (long)(b / g.dB) * g.sB;

  int kchunk = g.K;
  if (g.ksplit > 1) kchunk = (((g.K + g.ksplit - 1) / g.ksplit) + KS - 1) / KS * KS;
  const int kbeg = sp * kchunk;
  const int kend = min(g.K, kbeg + kchunk);

  // Three real products per complex product (Karatsuba): t1 = Re A Re B,
  // t2 = Im A Im B, t3 = (Re A + Im A)(Re B + Im B); Re C = t1 - t2, Im C = t3 - t1 - t2.
  // Its rounding error is bounded by a small multiple of eps |A| |B|, as for four.
  ACC t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      t1[i][j] = (ACC){0, 0, 0, 0};
      t2[i][j] = (ACC){0, 0, 0, 0};
      t3[i][j] = (ACC){0, 0, 0, 0};
    }

  // Group index gi = tid + 256 * r.  OPA = 0 (A column-major, contiguous in i): group
  // (i-block, k) with i-block fastest; OPA = 1 (A^H, contiguous in k): (k-block, i).
  // Columns known to be zero (GemmArgs::zrn) are not loaded: with OPA = 1 a group's i, and
  // with OPB = 0 a group's j, is the same for every k.
  bool za[GA], zb[GB];
#pragma unroll
  for (int r = 0; r < GA; ++r)
    za[r] = OPA == 1 && zero_col(g, b / g.kdiv, row0 + (tid + 256 * r) / (KS / VA));
#pragma unroll
  for (int r = 0; r < GB; ++r)
    zb[r] = OPB == 0 && g.zs > 0 && zero_col(g, b / g.kdiv, (col0 + (tid + 256 * r) / (KS / VB)) % (3 * g.zs));
  C ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < GA; ++r) {
      const int gi = tid + 256 * r;
#pragma unroll
      for (int q = 0; q < VA; ++q) {
        int i, k;
        if (OPA == 0) { i = row0 + (gi % (BM / VA)) * VA + q; k = k0 + gi / (BM / VA); }
        else { k = k0 + (gi % (KS / VA)) * VA + q; i = row0 + gi / (KS / VA); }
        C v = mk<R>(0, 0);
        if (i < g.M && k < kend && !za[r]) v = (OPA == 0) ? A[i + (long)k * g.lda] : A[k + (long)i * g.lda];
        ra[r * VA + q] = v;
      }
    }
#pragma unroll
    for (int r = 0; r < GB; ++r) {
      const int gi = tid + 256 * r;
#pragma unroll
      for (int q = 0; q < VB; ++q) {
        int j, k;
        if (OPB == 0) { k = k0 + (gi % (KS / VB)) * VB + q; j = col0 + gi / (KS / VB); }
        else { j = col0 + (gi % (BN / VB)) * VB + q; k = k0 + gi / (BN / VB); }
        C w = mk<R>(0, 0);
        if (j < g.N && k < kend && !zb[r]) w = (OPB == 0) ? B[k + (long)j * g.ldb] : B[j + (long)k * g.ldb];
        rb[r * VB + q] = w;
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < GA; ++r) {
      const int gi = tid + 256 * r;
#pragma unroll
      for (int q = 0; q < VA; ++q) {
        int ii, kk;
        if (OPA == 0) { ii = (gi % (BM / VA)) * VA + q; kk = gi / (BM / VA); }
        else { kk = (gi % (KS / VA)) * VA + q; ii = gi / (KS / VA); }
        Asr[kk][ii] = ra[r * VA + q].x;
        Asi[kk][ii] = OPA == 0 ? ra[r * VA + q].y : -ra[r * VA + q].y;
      }
    }
#pragma unroll
    for (int r = 0; r < GB; ++r) {
      const int gi = tid + 256 * r;
#pragma unroll
      for (int q = 0; q < VB; ++q) {
        int jj, kk;
        if (OPB == 0) { kk = (gi % (KS / VB)) * VB + q; jj = gi / (KS / VB); }
        else { jj = (gi % (BN / VB)) * VB + q; kk = gi / (BN / VB); }
        Bsr[kk][jj] = rb[r * VB + q].x;
        Bsi[kk][jj] = OPB == 0 ? rb[r * VB + q].y : -rb[r * VB + q].y;
      }
    }
  };

  auto compute = [&]() {
#pragma unroll
    for (int kk = 0; kk < KS / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      {
        R ar[2], ai[2], as[2], br[2], bi[2], bs[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          ar[x] = Asr[kr][wr * 32 + x * 16 + (lane & 15)];
          ai[x] = Asi[kr][wr * 32 + x * 16 + (lane & 15)];
          br[x] = Bsr[kr][wc * 32 + x * 16 + (lane & 15)];
          bi[x] = Bsi[kr][wc * 32 + x * 16 + (lane & 15)];
          as[x] = ar[x] + ai[x];
          bs[x] = br[x] + bi[x];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            t1[x][y] = mfma16(br[y], ar[x], t1[x][y]);
            t2[x][y] = mfma16(bi[y], ai[x], t2[x][y]);
            t3[x][y] = mfma16(bs[y], as[x], t3[x][y]);
          }
      }
    }
  };

  // One LDS stage; the next stage's global loads are in flight in registers while the
  // current stage is multiplied (two barriers per stage).  Many designs' kernels share the
  // GPU, and a tile's LDS decides how many workgroups fit on a CU beside the others: one
  // stage (21 KiB for 128 x 32 FP32 tiles instead of 43) keeps more of them resident,
  // which measured faster than two stages with one barrier each.
  if (kbeg < kend) {
    load(kbeg);
    store();
  }
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += KS) {
    const bool more = k0 + KS < kend;
    if (more) load(k0 + KS);
    compute();
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }

  // Epilogue.
  const bool part = g.ksplit > 1;
  C* Cb = part ? g.Cpart + ((long)sp * g.batch + b) * (long)g.M * g.N
               : g.Cm + (long)(b / g.dC) * g.sC;
  const long ldc = part ? g.M : g.ldc;
  const bool useBeta = !part && (g.beta.x != 0 || g.beta.y != 0);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wr * 32 + x * 16 + (lane & 15);
        // MFMA result layout (lane l, register r): FP32 holds row 4(l/16)+r, FP64 holds
        // row l/16 + 4r of the 16x16 block, column l%16 in both (here rows are C columns).
        const int col = col0 + wc * 32 + y * 16 + (sizeof(R) == 8 ? ((lane >> 4) + 4 * r) : (((lane >> 4) << 2) + r));
        if (row < g.M && col < g.N) {
          const C acc = mk<R>(t1[x][y][r] - t2[x][y][r], t3[x][y][r] - t1[x][y][r] - t2[x][y][r]);
          C v = cmul(g.alpha, acc);
          if (useBeta) v = cadd(v, cmul(g.beta, Cb[row + (long)col * ldc]));
          Cb[row + (long)col * ldc] = v;
        }
      }
}

// Real k-shared operators times complex blocks (OpArgs): one 64 x 64 output tile per
// workgroup of 4 waves, two real MFMA products per complex one (A Re B and A Im B), one LDS
// stage of KS = 8 with the next stage's global loads in flight.  The tiles of all the
// launch's products form one list: within a product the 64-row tiles of one (item, column
// tile) are consecutive, so they share that block's columns, and the list is dealt to
// the 8 XCDs in contiguous ranges (workgroups go to XCDs round-robin by linear id).  Only
// listed items have tiles, so converged k-points cost nothing and the work of every XCD
// is the same.
__device__ __forceinline__ long op_tiles(const OpSeg& s, int tm) {
  const int tn = (s.ncolk > 0 ? s.nb * s.ncolk + 63 : s.N + 63) / 64;
  return (long)tm * tn * (s.ncolk > 0 ? 1 : s.nb);
}

template <int KS>
__global__ __launch_bounds__(256, 3) void opgemm_kernel(OpArgs g) {
  constexpr int BM = 64, BN = 64;
  constexpr int RA = KS / 8, RB = KS / 4;  // per thread: RA row pairs of A, RB consecutive k of B
  __shared__ double As[KS][BM + 4], Bsr[KS][BN + 4], Bsi[KS][BN + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int tm = (g.M + BM - 1) / BM;
  const long c0 = op_tiles(g.seg[0], tm), c1 = g.nseg > 1 ? op_tiles(g.seg[1], tm) : 0;
  const long c2 = g.nseg > 2 ? op_tiles(g.seg[2], tm) : 0;
  long logical;
  {
    const long total = c0 + c1 + c2, lin = blockIdx.x;
    const long per = total / 8, rem = total % 8, xcd = lin % 8, idx = lin / 8;
    logical = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  }
  int si = 0;
  if (logical >= c0) {
    logical -= c0;
    si = 1;
    if (logical >= c1) {
      logical -= c1;
      si = 2;
    }
  }
  const OpSeg S = si == 0 ? g.seg[0] : (si == 1 ? g.seg[1] : g.seg[2]);
  const int ncols = S.ncolk > 0 ? S.nb * S.ncolk : S.N;
  const int tn = (ncols + BN - 1) / BN;
  const int ti = (int)(logical % tm);
  const long rest = logical / tm;
  const int tj = (int)(rest % tn), bat = (int)(rest / tn);
  const int row0 = ti * BM, col0 = tj * BN;
  const double2* B = S.B;
  double2* Cb = S.C;
  if (S.ncolk == 0) {
    const long it = S.bidx ? S.bidx[bat] : bat;
    B += it * S.sB;
    Cb += it * S.sC;
  }
  // where column j of this product is stored in B and in C
  const int kd = S.kdiv > 0 ? S.kdiv : 1;
  auto boff = [&](int j) -> long {
    if (S.ncolk == 0) return (long)j * S.ldb;
    const int e = S.bidx[j / S.ncolk];
    return (long)(e / kd) * S.sB + (long)((e % kd) * S.ncolk + j % S.ncolk) * S.ldb;
  };
  auto coff = [&](int j) -> long {
    if (S.ncolk == 0) return (long)j * S.ldc;
    const int e = S.bidx[j / S.ncolk];
    return (long)(e / kd) * S.sC + (long)((e % kd) * S.ncolk + j % S.ncolk) * S.ldc;
  };

  // staging: A 64 x KS (RA pairs of consecutive rows per thread, k = ak + 8 r), B KS x 64
  // (RB consecutive k of one column per thread); the thread's B column is fixed for the tile
  const int ai = (tid % 32) * 2, ak = tid / 32;
  const int bk = (tid % 4) * RB, bj = tid / 4;
  const bool bvalid = col0 + bj < ncols;
  const double2* bcol = B + (bvalid ? boff(col0 + bj) : 0);
  double ra[2 * RA];
  double2 rb[RB];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < RA; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int i = row0 + ai + q, k = k0 + ak + 8 * r;
        ra[2 * r + q] = (i < g.M && k < g.K) ? S.A[i + (long)k * g.lda] : 0.0;
      }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int k = k0 + bk + q;
      rb[q] = (bvalid && k < g.K) ? bcol[k] : make_double2(0, 0);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < RA; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) As[ak + 8 * r][ai + q] = ra[2 * r + q];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      Bsr[bk + q][bj] = rb[q].x;
      Bsi[bk + q][bj] = rb[q].y;
    }
  };
  typedef acc_t<double>::type ACC;
  ACC t1[2][2], t2[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      t1[x][y] = (ACC){0, 0, 0, 0};
      t2[x][y] = (ACC){0, 0, 0, 0};
    }
  load(0);
  store();
  __syncthreads();
  for (int k0 = 0; k0 < g.K; k0 += KS) {
    const bool more = k0 + KS < g.K;
    if (more) load(k0 + KS);
#pragma unroll
    for (int kk = 0; kk < KS / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double ar[2], br[2], bi[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        ar[x] = As[kr][wr * 32 + x * 16 + (lane & 15)];
        br[x] = Bsr[kr][wc * 32 + x * 16 + (lane & 15)];
        bi[x] = Bsi[kr][wc * 32 + x * 16 + (lane & 15)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          t1[x][y] = mfma16(br[y], ar[x], t1[x][y]);
          t2[x][y] = mfma16(bi[y], ar[x], t2[x][y]);
        }
    }
    __syncthreads();
    if (more) {
      store();
      __syncthreads();
    }
  }
  // epilogue: lane l, register r of a 16 x 16 block holds row l % 16, column l / 16 + 4 r
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int col = col0 + wc * 32 + y * 16 + (lane >> 4) + 4 * r;
      if (col >= ncols) continue;
      double2* cc = Cb + coff(col);
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int row = row0 + wr * 32 + x * 16 + (lane & 15);
        if (row < g.M) cc[row] = make_double2(t1[x][y][r], t2[x][y][r]);
      }
    }
}

int opgemm(const OpArgs& g, hipStream_t st) {
  if (g.nseg < 1 || g.nseg > 3 || g.M <= 0 || g.K <= 0) return (int)hipErrorInvalidValue;
  const int tm = (g.M + 63) / 64;
  long total = 0;
  for (int s = 0; s < g.nseg; ++s) {
    const OpSeg& q = g.seg[s];
    if (q.nb < 0 || (q.ncolk > 0 && !q.bidx)) return (int)hipErrorInvalidValue;
    const int ncols = q.ncolk > 0 ? q.nb * q.ncolk : q.N;
    total += (long)tm * ((ncols + 63) / 64) * (q.ncolk > 0 ? 1 : q.nb);
  }
  if (total == 0) return 0;
  if (total > 0x7fffffffL) return (int)hipErrorInvalidValue;
#define PHX_OP_LAUNCH(KSv)                                                                              \
  do {                                                                                                   \
    if (g.ev0)                                                                                           \
      hipExtLaunchKernelGGL(opgemm_kernel<KSv>, dim3((unsigned)total), dim3(256), 0, st, g.ev0, g.ev1, 0, g); \
    else hipLaunchKernelGGL(opgemm_kernel<KSv>, dim3((unsigned)total), dim3(256), 0, st, g);           \
  } while (0)
  PHX_OP_LAUNCH(8);  // a 16-deep stage measured slower
#undef PHX_OP_LAUNCH
  return (int)hipGetLastError();
}

// Tall-skinny products C = A W (beta = 0, alpha = 1) with K <= 64, N <= 16 NB: the
// subspace updates [S | KS | Omega S] C of the eigensolver.  Optionally output columns
// j >= csplit go to column j + cgap (two coefficient blocks, one pass over A).  W is staged in LDS once
// per workgroup; a wave takes ST stripes of 16 rows and, per stripe, issues the loads of
// all its A values (16 consecutive rows per load, every k) before the first product, so
// one stripe's whole row block is in flight at once.  Three real products per complex
// product (Karatsuba).
template <typename R, int NB, int ST>
__global__ __launch_bounds__(256, 3) void skinny_kernel(GemmArgs<R> g) {
  typedef C_t<R> C;
  typedef typename acc_t<R>::type ACC;
  constexpr int NC = 16 * NB;
  __shared__ R Wr[64][NC + 1], Wi[64][NC + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int b = g.bidx ? g.bidx[blockIdx.y / g.kdiv] * g.kdiv + blockIdx.y % g.kdiv : blockIdx.y;
  if (g.kact && !g.kact[b / g.kdiv]) return;  // whole workgroup: a converged k-point
  const C* A = g.A + (long)(b / g.dA) * g.sA;
  const C* W = g.B + (long)(b / g.dB) * g.sB;
  C* Cb = g.Cm + (long)(b / g.dC) * g.sC;
  for (int e = tid; e < 64 * NC; e += 256) {
    const int k = e & 63, j = e >> 6;
    C v = mk<R>(0, 0);
    if (k < g.K && j < g.N) v = W[k + (long)j * g.ldb];
    Wr[k][j] = v.x;
    Wi[k][j] = v.y;
  }
  __syncthreads();
  // the columns of A known to be zero (bit k: column k, the same in every wave), not loaded
  const unsigned long long zmask = __ballot(zero_col(g, b / g.kdiv, lane));
#pragma unroll 1
  for (int stripe = 0; stripe < ST; ++stripe) {
    const int i0 = blockIdx.x * 64 * ST + wave * 16 * ST + 16 * stripe;
    if (i0 >= g.M) break;
    const int i = i0 + li;
    ACC t1[NB], t2[NB], t3[NB];
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      t1[y] = (ACC){0, 0, 0, 0};
      t2[y] = (ACC){0, 0, 0, 0};
      t3[y] = (ACC){0, 0, 0, 0};
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {  // four quarters of the k range, 4 loads in flight each
      C av[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = 16 * h + 4 * q + lg;
        av[q] = (i < g.M && k < g.K && !((zmask >> k) & 1ull)) ? A[i + (long)k * g.lda] : mk<R>(0, 0);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // k >= K: A is zero there and W's rows are zero
        const int k = 16 * h + 4 * q + lg;
        const R ar = av[q].x, ai = av[q].y, as = ar + ai;
#pragma unroll
        for (int y = 0; y < NB; ++y) {
          const R br = Wr[k][16 * y + li], bi = Wi[k][16 * y + li];
          t1[y] = mfma16(br, ar, t1[y]);
          t2[y] = mfma16(bi, ai, t2[y]);
          t3[y] = mfma16(br + bi, as, t3[y]);
        }
      }
    }
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * y + (sizeof(R) == 8 ? (lg + 4 * r) : (4 * lg + r));
        const int cc = (g.csplit > 0 && col >= g.csplit) ? col + g.cgap : col;
        if (i < g.M && col < g.N)
          Cb[i + (long)cc * g.ldc] = mk<R>(t1[y][r] - t2[y][r], t3[y][r] - t1[y][r] - t2[y][r]);
      }
  }
}

// Products with few right-hand sides, C = alpha op(A) B + beta C with N <= 16 NB and
// op(B) = B: the steps of the triangular solves, bound by the one pass over A.  A goes
// from global memory straight into MFMA operand registers, 16 k at a time, with the
// next 16 in flight while the current ones are multiplied; B is staged in LDS 64 rows
// at a time.  Wave w computes rows 16 X w .. 16 X (w + 1) - 1 of the workgroup's 64 X.
// OPA = 1 (A^H, stored A contiguous in k): a lane reads four consecutive k of one
// column of the stored A, so inside a 16-deep group the k order is permuted, the same
// permutation for both operands.
template <typename R, int OPA, int NB, int X>
__global__ __launch_bounds__(256, 3) void nrhs_kernel(GemmArgs<R> g) {
  typedef C_t<R> C;
  typedef typename acc_t<R>::type ACC;
  constexpr bool K3 = sizeof(R) == 4;  // FP32: three real products per complex product
  constexpr int KC = 64;
  constexpr int NC = 16 * NB;
  // row pitch: lanes 16..31 read the next k row (OPA = 0) or the row four further
  // (OPA = 1); the pitch puts them on the other 16 of 32 banks
  constexpr int LDB = OPA == 0 ? 48 : (NC == 16 ? 20 : 36);
  __shared__ R Br[KC][LDB], Bi[KC][LDB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int b = blockIdx.y;
  if (g.kact && !g.kact[b / g.kdiv]) return;  // whole workgroup: a converged k-point
  const C* A = g.A + (long)(g.amap ? g.amap[b] : b / g.dA) * g.sA;
  const C* Bm = g.B + (long)(b / g.dB) * g.sB;
  C* Cb = g.Cm + (long)(b / g.dC) * g.sC;
  const int i0 = blockIdx.x * 64 * X + wave * 16 * X;

  ACC t1[X][NB], t2[X][NB], t3[X][NB];
#pragma unroll
  for (int x = 0; x < X; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y) {
      t1[x][y] = (ACC){0, 0, 0, 0};
      t2[x][y] = (ACC){0, 0, 0, 0};
      t3[x][y] = (ACC){0, 0, 0, 0};
    }
  // k of slot q of this lane inside a 16-deep group
  auto kof = [&](int q) { return OPA == 0 ? 4 * q + lg : 4 * lg + q; };
  auto loadA = [&](int k0, C (&v)[X][4]) {
#pragma unroll
    for (int x = 0; x < X; ++x) {
      const int i = i0 + 16 * x + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + kof(q);
        C a = mk<R>(0, 0);
        if (i < g.M && k < g.K) a = OPA == 0 ? A[i + (long)k * g.lda] : A[k + (long)i * g.lda];
        v[x][q] = a;
      }
    }
  };
  auto stageB = [&](int k0) {
    for (int e = tid; e < KC * NC; e += 256) {
      const int k = e % KC, j = e / KC;
      C v = mk<R>(0, 0);
      if (k0 + k < g.K && j < g.N) v = Bm[k0 + k + (long)j * g.ldb];
      Br[k][j] = v.x;
      Bi[k][j] = v.y;
    }
  };
  auto mult = [&](const C (&v)[X][4], int kl) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kl + kof(q);
      R ar[X], ai[X], as[X];
#pragma unroll
      for (int x = 0; x < X; ++x) {
        ar[x] = v[x][q].x;
        ai[x] = OPA == 0 ? v[x][q].y : -v[x][q].y;
        if (K3) as[x] = ar[x] + ai[x];
      }
#pragma unroll
      for (int y = 0; y < NB; ++y) {
        const R br = Br[k][16 * y + li], bi = Bi[k][16 * y + li];
#pragma unroll
        for (int x = 0; x < X; ++x) {
          if (K3) {
            const R bs = br + bi;  // in registers: a third LDS array would cost residency
            t1[x][y] = mfma16(br, ar[x], t1[x][y]);
            t2[x][y] = mfma16(bi, ai[x], t2[x][y]);
            t3[x][y] = mfma16(bs, as[x], t3[x][y]);
          } else {
            t1[x][y] = mfma16(br, ar[x], t1[x][y]);
            t3[x][y] = mfma16(bi, ar[x], t3[x][y]);
            t1[x][y] = mfma16(-bi, ai[x], t1[x][y]);
            t3[x][y] = mfma16(br, ai[x], t3[x][y]);
          }
        }
      }
    }
  };

  const int ng = (g.K + 15) / 16;
  C va[X][4], vb[X][4];
  loadA(0, va);
  for (int gi = 0; gi < ng; gi += 2) {
    if ((gi * 16) % KC == 0) {
      __syncthreads();
      stageB(gi * 16);
      __syncthreads();
    }
    if (gi + 1 < ng) loadA((gi + 1) * 16, vb);
    mult(va, (gi * 16) % KC);
    if (gi + 1 >= ng) break;
    if (gi + 2 < ng) loadA((gi + 2) * 16, va);
    mult(vb, ((gi + 1) * 16) % KC);
  }

  const bool useBeta = g.beta.x != 0 || g.beta.y != 0;
#pragma unroll
  for (int x = 0; x < X; ++x)
#pragma unroll
    for (int y = 0; y < NB; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = i0 + 16 * x + li;
        const int col = 16 * y + (sizeof(R) == 8 ? (lg + 4 * r) : (4 * lg + r));
        if (row < g.M && col < g.N) {
          const C acc = K3 ? mk<R>(t1[x][y][r] - t2[x][y][r], t3[x][y][r] - t1[x][y][r] - t2[x][y][r])
                           : mk<R>(t1[x][y][r], t3[x][y][r]);
          C v = cmul(g.alpha, acc);
          if (useBeta) v = cadd(v, cmul(g.beta, Cb[row + (long)col * g.ldc]));
          Cb[row + (long)col * g.ldc] = v;
        }
      }
}

template <typename R>
__global__ void zgemm_reduce_kernel(GemmArgs<R> g) {
  typedef C_t<R> C;
  const long MN = (long)g.M * g.N;
  const int b = g.bidx ? g.bidx[blockIdx.y / g.kdiv] * g.kdiv + blockIdx.y % g.kdiv : blockIdx.y;
  if (g.kact && !g.kact[b / g.kdiv]) return;
  C* Cb = g.Cm + (long)(b / g.dC) * g.sC;
  const bool useBeta = (g.beta.x != 0 || g.beta.y != 0);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < MN; e += (long)gridDim.x * blockDim.x) {
    const int row = (int)(e % g.M), col = (int)(e / g.M);
    C s = mk<R>(0, 0);
    for (int sp = 0; sp < g.ksplit; ++sp) s = cadd(s, g.Cpart[((long)sp * g.batch + b) * MN + e]);
    if (useBeta) s = cadd(s, cmul(g.beta, Cb[row + (long)col * g.ldc]));
    Cb[row + (long)col * g.ldc] = s;
  }
}

// One launch of kernel K on grid G with the arguments g; with g.ev0 set, the launch
// records g.ev0 / g.ev1 at the kernel's start and end.
#define PHX_LAUNCH(K, G)                                                          \
  do {                                                                            \
    if (g.ev0) hipExtLaunchKernelGGL(K, G, dim3(256), 0, st, g.ev0, g.ev1, 0, g); \
    else hipLaunchKernelGGL(K, G, dim3(256), 0, st, g);                          \
  } while (0)

template <typename R>
int zgemm(const GemmArgs<R>& g0, int opa, int opb, hipStream_t st) {
  GemmArgs<R> g = g0;
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return 0;
  if (g.dA <= 0) g.dA = 1;
  if (g.dB <= 0) g.dB = 1;
  if (g.dC <= 0) g.dC = 1;
  if (g.kdiv <= 0) g.kdiv = 1;
  if (g.ksplit < 1) g.ksplit = 1;
  if (g.K <= 0) {  // C = beta C
    g.ksplit = 1;
  }
  if (g.ksplit > 1) g.ev0 = g.ev1 = nullptr;  // two kernels: no single-kernel timing
  // Listed batch items only (tiled, tall-skinny and reduction kernels): the grid covers
  // nbat * kdiv items.
  if (g.bidx && g.nbat <= 0) return 0;
  const unsigned nbatch = g.bidx ? (unsigned)(g.nbat * g.kdiv) : (unsigned)g.batch;
  // Tall-skinny updates (the eigensolver's basis times a small coefficient matrix).
  if (opa == 0 && opb == 0 && !g.tri && !g.amap && g.ksplit == 1 && g.K <= 64 && g.N <= 64 &&
      (g.M >= 256 || g.csplit > 0) &&
      g.alpha.x == 1 && g.alpha.y == 0 && g.beta.x == 0 && g.beta.y == 0) {
    dim3 grid2((unsigned)((g.M + 64 * 4 - 1) / (64 * 4)), nbatch);
    if (g.N <= 16) PHX_LAUNCH((skinny_kernel<R, 1, 4>), grid2);
    else if (g.N <= 32) PHX_LAUNCH((skinny_kernel<R, 2, 4>), grid2);
    else if (g.N <= 48) PHX_LAUNCH((skinny_kernel<R, 3, 4>), grid2);
    else PHX_LAUNCH((skinny_kernel<R, 4, 4>), grid2);
    return (int)hipGetLastError();
  }
  if (g.csplit > 0) return (int)hipErrorInvalidValue;  // split output only in the tall-skinny kernel
  if (g.amap && g.ksplit > 1) return (int)hipErrorInvalidValue;
  // Few right-hand sides (N <= 32, B not transposed): one streaming pass over A (for
  // FP32 A^H with more than 256 rows the LDS-staged 128 x 32 tiles below read A faster).
  if (!g.tri && !g.bidx && !g.tiled && opb == 0 && g.ksplit == 1 && g.N <= 32 && g.K > 0 &&
      (opa == 0 || sizeof(R) == 8 || g.M <= 256)) {
    constexpr int X = 1;
    dim3 grid2((unsigned)((g.M + 64 * X - 1) / (64 * X)), (unsigned)g.batch);
    if (opa == 0) {
      if (g.N <= 16) PHX_LAUNCH((nrhs_kernel<R, 0, 1, X>), grid2);
      else PHX_LAUNCH((nrhs_kernel<R, 0, 2, X>), grid2);
    } else {
      if (g.N <= 16) PHX_LAUNCH((nrhs_kernel<R, 1, 1, X>), grid2);
      else PHX_LAUNCH((nrhs_kernel<R, 1, 2, X>), grid2);
    }
    return (int)hipGetLastError();
  }
  // Narrow outputs (N <= 32: triangular solves and updates with the s search
  // vectors) use 128 x 32 tiles; everything else 64 x 64.
  const bool narrow = !g.tri && g.N <= 32 && g.tiled != 2;
  const int BM = narrow ? 128 : 64, BN = narrow ? 32 : 64;
  long ntiles;
  const long tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  if (g.tri) ntiles = tm * (tm + 1) / 2;
  else ntiles = tm * tn;
  dim3 grid((unsigned)ntiles, nbatch, (unsigned)g.ksplit);
#define PHX_GEMM_LAUNCH(BMv, BNv, T)                                      \
  do {                                                                     \
    if (opa == 0 && opb == 0) PHX_LAUNCH((zgemm_kernel<R, 0, 0, BMv, BNv, T>), grid); \
    else if (opa == 0 && opb == 1) PHX_LAUNCH((zgemm_kernel<R, 0, 1, BMv, BNv, T>), grid); \
    else if (opa == 1 && opb == 0) PHX_LAUNCH((zgemm_kernel<R, 1, 0, BMv, BNv, T>), grid); \
    else PHX_LAUNCH((zgemm_kernel<R, 1, 1, BMv, BNv, T>), grid);            \
  } while (0)
  // The lower-triangular tile grid (Hermitian rank-k update of the Cholesky trailing
  // matrix) is its own instantiation.
  if (g.tri) {
    if (opa == 0 && opb == 1) PHX_LAUNCH((zgemm_kernel<R, 0, 1, 64, 64, 1>), grid);
    else return (int)hipErrorInvalidValue;
  } else if (narrow) {
    PHX_GEMM_LAUNCH(128, 32, 0);
  } else {
    PHX_GEMM_LAUNCH(64, 64, 0);
  }
#undef PHX_GEMM_LAUNCH
  if (g.ksplit > 1) {
    long MN = (long)g.M * g.N;
    unsigned nb = (unsigned)std::min<long>((MN + 255) / 256, 1024);
    hipLaunchKernelGGL((zgemm_reduce_kernel<R>), dim3(nb, nbatch), dim3(256), 0, st, g);
  }
  return (int)hipGetLastError();
}

template int zgemm<double>(const GemmArgs<double>&, int, int, hipStream_t);
template int zgemm<float>(const GemmArgs<float>&, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Cholesky of the 64x64 diagonal block at (j0, j0) of every matrix in a batch,
// in place (lower triangle), and Dinv = L_jj^{-1} (lower, 64x64, ld 64).
// A non-positive or non-finite pivot raises a flag and is replaced by 1 so the
// factorisation stays finite; the host turns the flag into an error.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(1024) void potrf_diag_kernel(C_t<R>* A, long lda, long sA, int j0,
                                                          C_t<R>* Dinv, long sD, int* flag) {
  typedef C_t<R> C;
  __shared__ C Ls[64][65];  // Ls[col][row]
  __shared__ C Xs[64][65];  // L^{-1}, Xs[col][row]
  __shared__ R pivs[64];
  const int tid = threadIdx.x;
  C* Ab = A + (long)blockIdx.x * sA + j0 + (long)j0 * lda;
  for (int e = tid; e < 4096; e += 1024) {
    const int i = e & 63, j = e >> 6;
    Ls[j][i] = (i >= j) ? Ab[i + (long)j * lda] : mk<R>(0, 0);
    Xs[j][i] = mk<R>(i == j ? (R)1 : (R)0, 0);
  }
  __syncthreads();
  // Right-looking: the pivot is read by every thread, column k is scaled, then the
  // trailing lower triangle takes the rank-1 update.  The factor's diagonal is kept
  // in pivs (the unscaled Ls[k][k] stays in place until the end).
  for (int k = 0; k < 64; ++k) {
    R d = Ls[k][k].x;
    const bool bad = !(d > 0) || !isfinite((double)d);
    if (bad) d = 1;
    const R piv = sqrt(d);
    if (tid == 0) {
      if (bad) atomicOr(flag, isfinite((double)Ls[k][k].x) ? PHX_FLAG_NOTPD : PHX_FLAG_NONFINITE);
      pivs[k] = piv;
    }
    if (tid > k && tid < 64) Ls[k][tid] = cscale(Ls[k][tid], (R)1 / piv);
    __syncthreads();
    for (int e = tid; e < 4096; e += 1024) {
      const int i = e & 63, j = e >> 6;
      if (j > k && i >= j) Ls[j][i] = csub(Ls[j][i], cmulc(Ls[k][i], Ls[k][j]));
    }
    __syncthreads();
  }
  if (tid < 64) Ls[tid][tid] = mk<R>(pivs[tid], 0);
  // Inverse of the lower factor by right-looking substitution on the identity:
  // row i of X is final once divided by the pivot; it then updates the rows below.
  for (int i = 0; i < 64; ++i) {
    if (tid <= i) Xs[tid][i] = cscale(Xs[tid][i], (R)1 / pivs[i]);
    __syncthreads();
    for (int e = tid; e < 4096; e += 1024) {
      const int r = e & 63, t = e >> 6;
      if (r > i && t <= i) Xs[t][r] = csub(Xs[t][r], cmul(Ls[i][r], Xs[t][i]));
    }
    __syncthreads();
  }
  for (int e = tid; e < 4096; e += 1024) {
    const int i = e & 63, j = e >> 6;
    if (i >= j) Ab[i + (long)j * lda] = Ls[j][i];
    Dinv[(long)blockIdx.x * sD + (long)(j0 >> 6) * 4096 + i + 64 * j] = (i >= j) ? Xs[j][i] : mk<R>(0, 0);
  }
}

template <typename R>
int potrf_diag(C_t<R>* A, long lda, long sA, int batch, int j0, C_t<R>* Dinv, long sD, int* flag,
               hipStream_t st) {
  hipLaunchKernelGGL((potrf_diag_kernel<R>), dim3(batch), dim3(1024), 0, st, A, lda, sA, j0, Dinv, sD, flag);
  return (int)hipGetLastError();
}
template int potrf_diag<double>(double2*, long, long, int, int, double2*, long, int*, hipStream_t);
template int potrf_diag<float>(float2*, long, long, int, int, float2*, long, int*, hipStream_t);

// ---------------------------------------------------------------------------
// Blocked right-looking Cholesky of a batch of n x n Hermitian matrices (n a
// multiple of 64; lower triangle used and overwritten by L), keeping the
// inverted diagonal blocks of L in Dinv (batch x n/64 blocks of 64x64).
// ---------------------------------------------------------------------------
#define PHX_HOOK_BEGIN(c) \
  if (hook) hook->begin(hook->user, (c))
#define PHX_HOOK_END(c, f, b) \
  if (hook) hook->end(hook->user, (c), (f), (b))
#define PHX_HOOK_KEV(c, f, b, g) \
  if (hook && hook->kev) hook->kev(hook->user, (c), (f), (b), &(g).ev0, &(g).ev1)

// Two-level blocking: 64-wide panels inside 256-wide column blocks.  Inside a
// column block each panel updates only the block's remaining columns; the rest of
// the trailing matrix receives one rank-256 Hermitian update per block, which
// reads and writes the trailing matrix a quarter as often as rank-64 updates.
template <typename R>
int potrf_batched(C_t<R>* A, int n, long lda, long sA, int batch, C_t<R>* Dinv, long sD, int* flag,
                  hipStream_t st, const ProfHook* hook) {
  typedef C_t<R> C;
  constexpr int NB = 256;
  const double cb = (double)sizeof(C);
  for (int J = 0; J < n; J += NB) {
    const int w = std::min(NB, n - J);
    for (int j0 = J; j0 < J + w; j0 += 64) {
      const int j = j0 / 64;
      PHX_HOOK_BEGIN(PROF_POTRF_DIAG);
      int e = potrf_diag<R>(A, lda, sA, batch, j0, Dinv, sD, flag, st);
      PHX_HOOK_END(PROF_POTRF_DIAG, batch * 8.0 * 64 * 64 * 64 / 6.0, batch * cb * (64.0 * 64 * 2));
      if (e) return e;
      const int rem = n - j0 - 64;
      if (rem <= 0) break;
      C* panel = A + (j0 + 64) + (long)j0 * lda;
      {  // panel <- panel * Dinv_j^H   (in place: one 64-wide column tile per row tile)
        GemmArgs<R> g{};
        g.M = rem; g.N = 64; g.K = 64; g.batch = batch;
        g.A = panel; g.lda = lda; g.sA = sA;
        g.B = Dinv + (long)j * 4096; g.ldb = 64; g.sB = sD;
        g.Cm = panel; g.ldc = lda; g.sC = sA;
        g.alpha = mk<R>(1, 0); g.beta = mk<R>(0, 0);
        PHX_HOOK_BEGIN(PROF_PANEL);
        e = zgemm<R>(g, 0, 1, st);
        PHX_HOOK_END(PROF_PANEL, batch * 8.0 * rem * 64 * 64 / 2.0, batch * cb * (2.0 * rem * 64));
        if (e) return e;
      }
      const int nin = J + w - j0 - 64;  // columns of this block right of the panel
      if (nin > 0) {  // block columns j0+64 .. J+w, every row below the panel's diagonal tile
        GemmArgs<R> g{};
        g.M = rem; g.N = nin; g.K = 64; g.batch = batch;
        g.A = panel; g.lda = lda; g.sA = sA;
        g.B = panel; g.ldb = lda; g.sB = sA;
        g.Cm = A + (j0 + 64) + (long)(j0 + 64) * lda; g.ldc = lda; g.sC = sA;
        g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
        PHX_HOOK_BEGIN(PROF_PANEL);
        e = zgemm<R>(g, 0, 1, st);
        PHX_HOOK_END(PROF_PANEL, batch * 8.0 * 64 * ((double)rem * nin - nin * (nin - 1) / 2.0),
                     batch * cb * (2.0 * rem * nin + rem * 64.0));
        if (e) return e;
      }
    }
    const int rem2 = n - J - w;
    if (rem2 > 0) {  // trailing lower tiles -= block block^H (rank w)
      C* blk = A + (J + w) + (long)J * lda;
      GemmArgs<R> g{};
      g.M = rem2; g.N = rem2; g.K = w; g.batch = batch; g.tri = 1;
      g.A = blk; g.lda = lda; g.sA = sA;
      g.B = blk; g.ldb = lda; g.sB = sA;
      g.Cm = A + (J + w) + (long)(J + w) * lda; g.ldc = lda; g.sC = sA;
      g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
      // algorithmic: rank-w update of the lower triangle (rem2(rem2+1)/2 entries), read+write once
      PHX_HOOK_KEV(PROF_HERK, batch * 8.0 * w * (double)rem2 * (rem2 + 1) / 2.0,
                   batch * cb * ((double)rem2 * (rem2 + 1) + (double)rem2 * w), g);
      const int e = zgemm<R>(g, 0, 1, st);
      if (e) return e;
    }
  }
  return 0;
}
template int potrf_batched<double>(double2*, int, long, long, int, double2*, long, int*, hipStream_t,
                                   const ProfHook*);
template int potrf_batched<float>(float2*, int, long, long, int, float2*, long, int*, hipStream_t,
                                  const ProfHook*);

// ---------------------------------------------------------------------------
// Triangular solves with few right-hand sides (nc <= 32), one diagonal
// super-block of T <= WS/64 tiles per launch, one workgroup per matrix:
//   LOWER (L Z = B):    for t = 0..T-1:  Z_t = Dinv_t B_t;    B_u -= L_ut Z_t  (u > t)
//   UPPER (L^H Y = Z):  for t = T-1..0:  Y_t = Dinv_t^H Z_t;  Z_u -= L_tu^H Y_t (u < t)
// The super-block's right-hand side (rows J0 .. J0 + 64T of Bin) is held in LDS;
// the solution rows go to X.  The rest of the solve is a GEMM per super-block.
// Sixteen waves: waves 0-3 compute the diagonal tile's 16-row stripes, then every wave
// takes update stripes; MFMA k-index mapping: k = 4 ks + lane/16 when
// the operand is read down columns (coalesced over rows), k = 16 (lane/16) + ks
// when it is read along columns of L (each lane walks contiguous memory).
// ---------------------------------------------------------------------------
template <typename R, bool LOWER, int WS>
__global__ __launch_bounds__(1024) void trsv_block_kernel(const C_t<R>* L, long lda, long sL, const C_t<R>* Dinv,
                                                         long sD, const C_t<R>* Bin, long ldb, long sB, C_t<R>* X,
                                                         long ldx, long sX, int J0, int T, int nc) {
  typedef C_t<R> C;
  typedef typename acc_t<R>::type ACC;
  __shared__ R Sr[WS][32], Si[WS][32];
  // column swizzle by row parity: the four rows one MFMA operand read touches fall
  // in two different bank halves
#define SW(row, col) ((col) ^ (((row) & 1) << 4))
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const long b = blockIdx.x;
  const C* Lb = L + b * sL;
  const C* Db = Dinv + b * sD;
  C* Xb = X + b * sX;
  const int rows = 64 * T;
  for (int e = tid; e < rows * 32; e += 1024) {
    const int r = e % rows, c = e / rows;
    C v = mk<R>(0, 0);
    if (c < nc) v = Bin[b * sB + (J0 + r) + (long)c * ldb];
    Sr[r][SW(r, c)] = v.x;
    Si[r][SW(r, c)] = v.y;
  }
  __syncthreads();
  auto colmap = [&](int r) { return sizeof(R) == 8 ? (lg + 4 * r) : (4 * lg + r); };
  for (int step = 0; step < T; ++step) {
    const int t = LOWER ? step : T - 1 - step;
    const int tb = 64 * t;
    ACC cr[2], ci[2];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cr[y] = (ACC){0, 0, 0, 0};
      ci[y] = (ACC){0, 0, 0, 0};
    }
    if (wave < 4) {  // diagonal tile: rows 16 wave .. +16 of Dinv_t (or Dinv_t^H) times the tile's rhs
      const C* Dt = Db + (long)((J0 >> 6) + t) * 4096;
      const int i = 16 * wave + li;
      C av[16];  // all 16 operand loads in flight before the first product
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const int k = LOWER ? 4 * ks + lg : 16 * lg + ks;
        av[ks] = LOWER ? Dt[i + 64 * k] : cconj(Dt[k + 64 * i]);
      }
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const int k = LOWER ? 4 * ks + lg : 16 * lg + ks;
        const C a = av[ks];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int col = 16 * y + li, row = tb + k;
          const R br = Sr[row][SW(row, col)], bi = Si[row][SW(row, col)];
          cr[y] = mfma16(br, a.x, cr[y]);
          ci[y] = mfma16(bi, a.x, ci[y]);
          cr[y] = mfma16(-bi, a.y, cr[y]);
          ci[y] = mfma16(br, a.y, ci[y]);
        }
      }
    }
    __syncthreads();
    if (wave < 4) {
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = tb + 16 * wave + li, col = 16 * y + colmap(r);
          Sr[row][SW(row, col)] = cr[y][r];
          Si[row][SW(row, col)] = ci[y][r];
          if (col < nc) Xb[(J0 + row) + (long)col * ldx] = mk<R>(cr[y][r], ci[y][r]);
        }
    }
    __syncthreads();
    const int nu = LOWER ? T - 1 - t : t;
    for (int q = wave; q < 4 * nu; q += 16) {
      const int u = LOWER ? t + 1 + q / 4 : q / 4;
      const int r0 = 64 * u + 16 * (q % 4);
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        cr[y] = (ACC){0, 0, 0, 0};
        ci[y] = (ACC){0, 0, 0, 0};
      }
      C av[16];
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const int k = LOWER ? 4 * ks + lg : 16 * lg + ks;
        av[ks] = LOWER ? Lb[(J0 + r0 + li) + (long)(J0 + tb + k) * lda]
                       : cconj(Lb[(J0 + tb + k) + (long)(J0 + r0 + li) * lda]);
      }
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const int k = LOWER ? 4 * ks + lg : 16 * lg + ks;
        const C a = av[ks];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int col = 16 * y + li, row = tb + k;
          const R br = Sr[row][SW(row, col)], bi = Si[row][SW(row, col)];
          cr[y] = mfma16(br, a.x, cr[y]);
          ci[y] = mfma16(bi, a.x, ci[y]);
          cr[y] = mfma16(-bi, a.y, cr[y]);
          ci[y] = mfma16(br, a.y, ci[y]);
        }
      }
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + li, col = 16 * y + colmap(r);
          Sr[row][SW(row, col)] -= cr[y][r];
          Si[row][SW(row, col)] -= ci[y][r];
        }
    }
    __syncthreads();
  }
#undef SW
}

// The block columns below each diagonal super-block copied, conjugate-transposed, into
// the (otherwise unused) upper triangle: A[c][r] = conj(L[r][c]) for c in super-block J
// and r >= the end of J.  The forward solve then reads them as the backward solve reads
// the factor's row blocks, one contiguous column of the copy per output row.
template <typename R, int WS>
__global__ __launch_bounds__(256) void sb_transpose_kernel(C_t<R>* L, int n, long lda, long sL) {
  typedef C_t<R> C;
  __shared__ C tile[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int lim = min(n, (c0 / WS + 1) * WS);  // first row below the super-block of column c0
  if (r0 < lim || r0 >= n || c0 >= n) return;
  C* A = L + (long)blockIdx.z * sL;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + tx, c = c0 + k;
    tile[k][tx] = (r < n && c < n) ? A[r + (long)c * lda] : mk<R>(0, 0);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + tx, r = r0 + k;
    if (r < n && c < n) {
      const C v = tile[tx][k];
      A[c + (long)r * lda] = mk<R>(v.x, -v.y);
    }
  }
}

// Seeds of the super-block inversion, one workgroup row per (matrix, super-block) item
// b = f nsb + J: T_b = the lower triangle of the diagonal super-block L_JJ (zero above
// the diagonal and beyond the matrix), X_b = the inverted 64 x 64 diagonal blocks from
// the factorisation on its diagonal, zero elsewhere.  Both WS x WS, ld WS, stride WS^2.
template <typename R, int WS>
__global__ __launch_bounds__(256) void sb_seed_kernel(const C_t<R>* L, int n, long lda, long sL, int nsb,
                                                      const C_t<R>* Dinv, long sD, C_t<R>* T, C_t<R>* X) {
  typedef C_t<R> C;
  const long e = blockIdx.x * 256L + threadIdx.x;  // element r + c WS of the block
  const int b = blockIdx.y, f = b / nsb, J0 = (b % nsb) * WS;
  const int r = (int)(e % WS), c = (int)(e / WS);
  C tv = mk<R>(0, 0), xv = mk<R>(0, 0);
  if (J0 + r < n && J0 + c < n) {
    if (r >= c) tv = L[(long)f * sL + (J0 + r) + (long)(J0 + c) * lda];
    if (r / 64 == c / 64) xv = Dinv[(long)f * sD + (long)((J0 + r) / 64) * 4096 + (r % 64) + (c % 64) * 64];
  }
  T[(long)b * WS * WS + e] = tv;
  X[(long)b * WS * WS + e] = xv;
}

// Explicit inverses of the diagonal super-blocks of a batch of Cholesky factors
// (WS x WS blocks, ld WS, nsb = ceil(n / WS) per matrix, batch stride nsb WS^2), by
// recursive doubling from the factorisation's inverted 64 x 64 diagonal blocks: for a
// lower-triangular [[L11, 0], [L21, L22]] the inverse is [[X11, 0], [-X22 L21 X11, X22]]
// with X11, X22 the inverses of the halves.  Every (h, t) step (halves of order h = 64,
// 128, ..; pair t of the super-block) is two GEMMs batched over all super-blocks of all
// matrices, so the inversion runs on the matrix cores in large launches.  With the
// inverses every step of a narrow solve is a GEMM (no sequential dependency inside a
// super-block).  work: batch nsb (WS^2 + WS^2 / 4) elements.
template <typename R>
int sb_inverse_batched(C_t<R>* L, int n, long lda, long sL, int batch, const C_t<R>* Dinv, long sD,
                       C_t<R>* SBinv, C_t<R>* work, hipStream_t st) {
  constexpr int WS = sizeof(R) == 4 ? 256 : 128;
  const int nsb = (n + WS - 1) / WS;
  const int B = batch * nsb;
  const long S2 = (long)WS * WS;
  C_t<R>* T = work;
  C_t<R>* W = work + (long)B * S2;
  hipLaunchKernelGGL((sb_seed_kernel<R, WS>), dim3((unsigned)(S2 / 256), (unsigned)B), dim3(256), 0, st,
                     (const C_t<R>*)L, n, lda, sL, nsb, Dinv, sD, T, SBinv);
  int e = (int)hipGetLastError();
  if (e) return e;
  for (int h = 64; h < WS; h *= 2)
    for (int t = 0; t < WS / (2 * h); ++t) {
      const long o11 = (long)(2 * t * h) * (WS + 1);  // top-left of the pair's first half
      const long o21 = o11 + h;                       // its block below
      const long o22 = o11 + (long)h * (WS + 1);      // the second half
      {  // W = L21 X11
        GemmArgs<R> g{};
        g.M = h; g.N = h; g.K = h; g.batch = B;
        g.A = T + o21; g.lda = WS; g.sA = S2;
        g.B = SBinv + o11; g.ldb = WS; g.sB = S2;
        g.Cm = W; g.ldc = h; g.sC = (long)h * h;
        g.alpha = mk<R>(1, 0); g.beta = mk<R>(0, 0);
        if ((e = zgemm<R>(g, 0, 0, st))) return e;
      }
      {  // X21 = -X22 W
        GemmArgs<R> g{};
        g.M = h; g.N = h; g.K = h; g.batch = B;
        g.A = SBinv + o22; g.lda = WS; g.sA = S2;
        g.B = W; g.ldb = h; g.sB = (long)h * h;
        g.Cm = SBinv + o21; g.ldc = WS; g.sC = S2;
        g.alpha = mk<R>(-1, 0); g.beta = mk<R>(0, 0);
        if ((e = zgemm<R>(g, 0, 0, st))) return e;
      }
    }
  const unsigned nt = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL((sb_transpose_kernel<R, WS>), dim3(nt, nt, batch), dim3(256), 0, st, L, n, lda, sL);
  return (int)hipGetLastError();
}
template int sb_inverse_batched<double>(double2*, int, long, long, int, const double2*, long, double2*, double2*,
                                        hipStream_t);
template int sb_inverse_batched<float>(float2*, int, long, long, int, const float2*, long, float2*, float2*,
                                       hipStream_t);

// Narrow solve with the super-block inverses: per super-block one GEMM with the inverse
// (or its conjugate transpose) and one GEMM for the rows beyond it.
template <typename R>
int potrs_sbinv(const C_t<R>* L, int n, long lda, long sL, int batch, const C_t<R>* SBinv, C_t<R>* B, long ldb,
                long sB, C_t<R>* Z, long ldz, long sZ, int nc, hipStream_t st, const ProfHook* hook,
                const int* kact, const int* fmap, int nacc) {
  constexpr int WS = sizeof(R) == 4 ? 256 : 128;
  const double cb = (double)sizeof(C_t<R>);
  const int nsb = (n + WS - 1) / WS;
  const long sI = (long)nsb * WS * WS;
  const double na = nacc > 0 ? nacc : batch;  // right-hand-side blocks counted as work
  int e;
  for (int sbi = 0; sbi < nsb; ++sbi) {  // forward: L Z = B
    const int J0 = sbi * WS, w = std::min(WS, n - J0);
    {
      GemmArgs<R> g{};
      g.M = w; g.N = nc; g.K = w; g.batch = batch; g.kact = kact;
      g.A = SBinv + (long)sbi * WS * WS; g.lda = WS; g.sA = sI; g.amap = fmap;
      g.B = B + J0; g.ldb = ldb; g.sB = sB;
      g.Cm = Z + J0; g.ldc = ldz; g.sC = sZ;
      g.alpha = mk<R>(1, 0); g.beta = mk<R>(0, 0);
      PHX_HOOK_KEV(PROF_SOLVE_DIAG, na * 8.0 * w * (w + 64) / 2.0 * nc, na * cb * (w * (w + 64) / 2.0 + 2.0 * w * nc), g);
      e = zgemm<R>(g, 0, 0, st);
      if (e) return e;
    }
    const int rem = n - J0 - w;
    if (rem > 0) {
      GemmArgs<R> g{};
      g.M = rem; g.N = nc; g.K = w; g.batch = batch; g.kact = kact;
      // the conjugate-transposed copy of the block column (rows J0..J0+w, columns beyond)
      g.A = L + J0 + (long)(J0 + w) * lda; g.lda = lda; g.sA = sL; g.amap = fmap;
      g.tiled = sizeof(R) == 4;  // every FP32 update step on the one tiled A^H kernel
      g.B = Z + J0; g.ldb = ldz; g.sB = sZ;
      g.Cm = B + J0 + w; g.ldc = ldb; g.sC = sB;
      g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
      PHX_HOOK_KEV(PROF_SOLVE_UPD, na * 8.0 * rem * w * nc, na * cb * ((double)rem * w + 2.0 * rem * nc), g);
      e = zgemm<R>(g, 1, 0, st);
      if (e) return e;
    }
  }
  for (int sbi = nsb - 1; sbi >= 0; --sbi) {  // backward: L^H Y = Z, Y into B
    const int J0 = sbi * WS, w = std::min(WS, n - J0);
    {
      GemmArgs<R> g{};
      g.M = w; g.N = nc; g.K = w; g.batch = batch; g.kact = kact;
      g.A = SBinv + (long)sbi * WS * WS; g.lda = WS; g.sA = sI; g.amap = fmap;  // op = C: inverse of L_JJ^H
      g.B = Z + J0; g.ldb = ldz; g.sB = sZ;
      g.Cm = B + J0; g.ldc = ldb; g.sC = sB;
      g.alpha = mk<R>(1, 0); g.beta = mk<R>(0, 0);
      PHX_HOOK_KEV(PROF_SOLVE_DIAG, na * 8.0 * w * (w + 64) / 2.0 * nc, na * cb * (w * (w + 64) / 2.0 + 2.0 * w * nc), g);
      e = zgemm<R>(g, 1, 0, st);
      if (e) return e;
    }
    if (J0 > 0) {
      GemmArgs<R> g{};
      g.M = J0; g.N = nc; g.K = w; g.batch = batch; g.kact = kact;
      g.A = L + J0; g.lda = lda; g.sA = sL; g.amap = fmap;  // rows J0..J0+w, cols 0..J0-1; op = C
      g.tiled = sizeof(R) == 4;
      g.B = B + J0; g.ldb = ldb; g.sB = sB;
      g.Cm = Z; g.ldc = ldz; g.sC = sZ;
      g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
      PHX_HOOK_KEV(PROF_SOLVE_UPD, na * 8.0 * J0 * w * nc, na * cb * ((double)J0 * w + 2.0 * J0 * nc), g);
      e = zgemm<R>(g, 1, 0, st);
      if (e) return e;
    }
  }
  return 0;
}

// Narrow solve (nc <= 32): super-block kernels plus one GEMM per super-block.
template <typename R>
int potrs_narrow(const C_t<R>* L, int n, long lda, long sL, int batch, const C_t<R>* Dinv, long sD, C_t<R>* B,
                 long ldb, long sB, C_t<R>* Z, long ldz, long sZ, int nc, hipStream_t st, const ProfHook* hook) {
  constexpr int WS = sizeof(R) == 4 ? 256 : 128;
  const double cb = (double)sizeof(C_t<R>);
  const int nsb = (n + WS - 1) / WS;
  int e;
  for (int sbi = 0; sbi < nsb; ++sbi) {  // forward: L Z = B
    const int J0 = sbi * WS, w = std::min(WS, n - J0), T = w / 64;
    PHX_HOOK_BEGIN(PROF_TRSM_DIAG);
    hipLaunchKernelGGL((trsv_block_kernel<R, true, WS>), dim3(batch), dim3(1024), 0, st, L, lda, sL, Dinv, sD, B,
                       ldb, sB, Z, ldz, sZ, J0, T, nc);
    PHX_HOOK_END(PROF_TRSM_DIAG, batch * 8.0 * w * (w + 64) / 2.0 * nc, batch * cb * (w * (w + 64) / 2.0 + 2.0 * w * nc));
    if ((e = (int)hipGetLastError())) return e;
    const int rem = n - J0 - w;
    if (rem > 0) {
      GemmArgs<R> g{};
      g.M = rem; g.N = nc; g.K = w; g.batch = batch;
      g.A = L + (J0 + w) + (long)J0 * lda; g.lda = lda; g.sA = sL;
      g.B = Z + J0; g.ldb = ldz; g.sB = sZ;
      g.Cm = B + J0 + w; g.ldc = ldb; g.sC = sB;
      g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
      PHX_HOOK_BEGIN(PROF_TRSM_UPDATE);
      e = zgemm<R>(g, 0, 0, st);
      PHX_HOOK_END(PROF_TRSM_UPDATE, batch * 8.0 * rem * w * nc, batch * cb * ((double)rem * w + 2.0 * rem * nc));
      if (e) return e;
    }
  }
  for (int sbi = nsb - 1; sbi >= 0; --sbi) {  // backward: L^H Y = Z, Y into B
    const int J0 = sbi * WS, w = std::min(WS, n - J0), T = w / 64;
    PHX_HOOK_BEGIN(PROF_TRSM_DIAG);
    hipLaunchKernelGGL((trsv_block_kernel<R, false, WS>), dim3(batch), dim3(1024), 0, st, L, lda, sL, Dinv, sD, Z,
                       ldz, sZ, B, ldb, sB, J0, T, nc);
    PHX_HOOK_END(PROF_TRSM_DIAG, batch * 8.0 * w * (w + 64) / 2.0 * nc, batch * cb * (w * (w + 64) / 2.0 + 2.0 * w * nc));
    if ((e = (int)hipGetLastError())) return e;
    if (J0 > 0) {
      GemmArgs<R> g{};
      g.M = J0; g.N = nc; g.K = w; g.batch = batch;
      g.A = L + J0; g.lda = lda; g.sA = sL;  // rows J0..J0+w, cols 0..J0-1; op = C
      g.B = B + J0; g.ldb = ldb; g.sB = sB;
      g.Cm = Z; g.ldc = ldz; g.sC = sZ;
      g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
      PHX_HOOK_BEGIN(PROF_TRSM_UPDATE);
      e = zgemm<R>(g, 1, 0, st);
      PHX_HOOK_END(PROF_TRSM_UPDATE, batch * 8.0 * J0 * w * nc, batch * cb * ((double)J0 * w + 2.0 * J0 * nc));
      if (e) return e;
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Solve (L L^H) Y = B for a batch of factors from potrf_batched; B is n x nc
// (ld ldb, batch stride sB), Z is a work buffer of the same shape.  The result
// overwrites B.  Every block step is a GEMM with an inverted diagonal block.
// ---------------------------------------------------------------------------
template <typename R>
int potrs_batched(const C_t<R>* L, int n, long lda, long sL, int batch, const C_t<R>* Dinv, long sD,
                  C_t<R>* B, long ldb, long sB, C_t<R>* Z, long ldz, long sZ, int nc, hipStream_t st,
                  const ProfHook* hook, const C_t<R>* sbinv, const int* kact, const int* fmap, int nacc) {
  if (nc <= 32 && sbinv)
    return potrs_sbinv<R>(L, n, lda, sL, batch, sbinv, B, ldb, sB, Z, ldz, sZ, nc, st, hook, kact, fmap, nacc);
  if (fmap) return (int)hipErrorInvalidValue;  // shared factors only with the super-block inverses
  if (nc <= 32) return potrs_narrow<R>(L, n, lda, sL, batch, Dinv, sD, B, ldb, sB, Z, ldz, sZ, nc, st, hook);
  const int T = n / 64;
  const double cb = (double)sizeof(C_t<R>);
  int e;
  for (int j = 0; j < T; ++j) {  // forward: L Z = B
    const int j0 = j * 64;
    {
      GemmArgs<R> g{};
      g.M = 64; g.N = nc; g.K = 64; g.batch = batch;
      g.A = Dinv + (long)j * 4096; g.lda = 64; g.sA = sD;
      g.B = B + j0; g.ldb = ldb; g.sB = sB;
      g.Cm = Z + j0; g.ldc = ldz; g.sC = sZ;
      g.alpha = mk<R>(1, 0); g.beta = mk<R>(0, 0);
      PHX_HOOK_BEGIN(PROF_TRSM_DIAG);
      e = zgemm<R>(g, 0, 0, st);
      PHX_HOOK_END(PROF_TRSM_DIAG, batch * 8.0 * 64 * 64 * nc / 2, batch * cb * (64.0 * 64 / 2 + 2.0 * 64 * nc));
      if (e) return e;
    }
    if (j0 + 64 < n) {
      GemmArgs<R> g{};
      g.M = n - j0 - 64; g.N = nc; g.K = 64; g.batch = batch;
      g.A = L + (j0 + 64) + (long)j0 * lda; g.lda = lda; g.sA = sL;
      g.B = Z + j0; g.ldb = ldz; g.sB = sZ;
      g.Cm = B + j0 + 64; g.ldc = ldb; g.sC = sB;
      g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
      PHX_HOOK_BEGIN(PROF_TRSM_UPDATE);
      e = zgemm<R>(g, 0, 0, st);
      PHX_HOOK_END(PROF_TRSM_UPDATE, batch * 8.0 * g.M * 64 * nc, batch * cb * ((double)g.M * 64 + 2.0 * g.M * nc));
      if (e) return e;
    }
  }
  for (int j = T - 1; j >= 0; --j) {  // backward: L^H Y = Z, Y into B
    const int j0 = j * 64;
    {
      GemmArgs<R> g{};
      g.M = 64; g.N = nc; g.K = 64; g.batch = batch;
      g.A = Dinv + (long)j * 4096; g.lda = 64; g.sA = sD;
      g.B = Z + j0; g.ldb = ldz; g.sB = sZ;
      g.Cm = B + j0; g.ldc = ldb; g.sC = sB;
      g.alpha = mk<R>(1, 0); g.beta = mk<R>(0, 0);
      PHX_HOOK_BEGIN(PROF_TRSM_DIAG);
      e = zgemm<R>(g, 1, 0, st);
      PHX_HOOK_END(PROF_TRSM_DIAG, batch * 8.0 * 64 * 64 * nc / 2, batch * cb * (64.0 * 64 / 2 + 2.0 * 64 * nc));
      if (e) return e;
    }
    if (j0 > 0) {
      GemmArgs<R> g{};
      g.M = j0; g.N = nc; g.K = 64; g.batch = batch;
      g.A = L + j0; g.lda = lda; g.sA = sL;  // rows j0..j0+63, cols 0..j0-1; op = C
      g.B = B + j0; g.ldb = ldb; g.sB = sB;
      g.Cm = Z; g.ldc = ldz; g.sC = sZ;
      g.alpha = mk<R>(-1, 0); g.beta = mk<R>(1, 0);
      PHX_HOOK_BEGIN(PROF_TRSM_UPDATE);
      e = zgemm<R>(g, 1, 0, st);
      PHX_HOOK_END(PROF_TRSM_UPDATE, batch * 8.0 * g.M * 64 * nc, batch * cb * ((double)g.M * 64 + 2.0 * g.M * nc));
      if (e) return e;
    }
  }
  return 0;
}
template int potrs_batched<double>(const double2*, int, long, long, int, const double2*, long, double2*, long,
                                   long, double2*, long, long, int, hipStream_t, const ProfHook*, const double2*,
                                   const int*, const int*, int);
template int potrs_batched<float>(const float2*, int, long, long, int, const float2*, long, float2*, long,
                                  long, float2*, long, long, int, hipStream_t, const ProfHook*, const float2*,
                                  const int*, const int*, int);

}  // namespace phx
