// Internal interfaces between the phx kernels and the host runtime.
#pragma once
#include <algorithm>

#include "phx_common.h"

namespace phx {

// Batched complex GEMM: C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b], column-major.
// Operand X of batch item b starts at X + (b / dX) * sX (dX >= 1; sX = 0 shares it).
// tri = 1: only the lower-triangular 64x64 tiles of a square M x M output are computed.
// ksplit > 1: the K range is split over gridDim.z, partial products go to Cpart
// ([ksplit][batch][M*N]) and a second kernel sums them in a fixed order.
template <typename R>
struct GemmArgs {
  int M, N, K;
  int batch;
  const C_t<R>* A; long lda, sA; int dA;
  const C_t<R>* B; long ldb, sB; int dB;
  C_t<R>* Cm; long ldc, sC; int dC;
  C_t<R> alpha, beta;
  int tri;
  const int* kact;  // optional device mask: batch item b is skipped when kact[b / kdiv] == 0
  int kdiv;
  int ksplit;
  C_t<R>* Cpart;
  int csplit, cgap;  // tall-skinny only: output column j >= csplit (if > 0) is stored at j + cgap
  const int* amap;   // optional device map: batch item b reads A item amap[b] (instead of b / dA)
  hipEvent_t ev0, ev1;  // optional: recorded at the start and the end of the (single) kernel's execution
  int tiled;            // 1: always the LDS-tiled kernel, never the streaming few-RHS one; 2: and always 64 x 64 tiles
  // optional device list: only nbat * kdiv batch items run, grid item i being batch item
  // bidx[i / kdiv] * kdiv + i % kdiv (tiled, tall-skinny and split-K reduction kernels)
  const int* bidx;
  int nbat;
  // optional: columns of an eigensolver basis [X W P] (3 zs columns) that are known to be
  // zero, whose loads are skipped (the result is the same: the data is zero).  Column
  // c >= zs of k-point b / kdiv is zero when zfirst is set (W and P before the first
  // step) or when zrn[(b / kdiv) zs + c % zs] is below ztol (c % zs < znb) or zgtol (the
  // soft-locking test of the residual kernel, which zeroed those columns).  Used by the
  // tiled kernel for the columns of A^H (OPA = 1) and of B (OPB = 0, columns taken modulo
  // 3 zs) and by the tall-skinny kernel for the columns of A; the other kernels load them.
  const double* zrn;
  double ztol, zgtol;
  int zs, znb, zfirst;
};

// The zero-column test of GemmArgs (false without zrn).
template <typename R>
__device__ __forceinline__ bool zero_col(const GemmArgs<R>& g, int kpt, int c) {
  if (!g.zrn || c < g.zs || c >= 3 * g.zs) return false;
  if (g.zfirst) return true;
  const int j = c % g.zs;
  return g.zrn[(long)kpt * g.zs + j] < (j < g.znb ? g.ztol : g.zgtol);
}

template <typename R>
int zgemm(const GemmArgs<R>& g, int opa, int opb, hipStream_t st);

// Products of k-shared real operators with complex blocks, C = A B (the matrix-free
// operator products in the paired basis), up to three of them in one launch.  A: M x K
// real, column-major (ld lda), shared by every batch item of its product.  Batched form
// (ncolk == 0): item b of the product has B at B + it * sB (K x N, ld ldb) and C at
// C + it * sC (M x N, ld ldc), it = bidx[b] when bidx is given (the listed items only),
// else b, for b < nb.  Column-listed form (ncolk > 0): one product over the nb * ncolk
// columns of the listed entries packed side by side (so the 64-column tiles are full),
// column j being column q = j % ncolk of entry e = bidx[j / ncolk], which is group
// g = e % kdiv of item it = e / kdiv (kdiv >= 1): stored in B at
// it * sB + (g * ncolk + q) * ldb and in C at it * sC + (g * ncolk + q) * ldc.
struct OpSeg {
  const double* A;
  const double2* B;
  double2* C;
  long ldb, sB, ldc, sC;
  int N, nb, ncolk;
  const int* bidx;
  int kdiv;
};
struct OpArgs {
  OpSeg seg[3];
  int nseg, M, K;
  long lda;
  hipEvent_t ev0, ev1;  // optional: recorded at the kernel's start and end
};
int opgemm(const OpArgs& g, hipStream_t st);

// Optional timing hook around kernel launches (class id, algorithmic flops/bytes).
enum ProfClass {
  PROF_POTRF_DIAG = 0,
  PROF_PANEL,
  PROF_HERK,
  PROF_TRSM_DIAG,
  PROF_TRSM_UPDATE,
  PROF_SOLVE_UPD,   // block-column / row-block steps of the super-block solves (one kernel)
  PROF_SOLVE_DIAG,  // inverse-diagonal-block steps of the super-block solves
  PROF_SBINV,      // inverses of the factor's diagonal super-blocks
  PROF_NCLASS_DENSE
};
// begin/end: events recorded on the stream around a group of launches.  kev: two events
// for one kernel launch to record at its start and end (hipExtLaunchKernelGGL), with the
// launch's algorithmic work; null events when timing is off.
struct ProfHook {
  void (*begin)(void* user, int cls);
  void (*end)(void* user, int cls, double flops, double bytes);
  void (*kev)(void* user, int cls, double flops, double bytes, hipEvent_t* a, hipEvent_t* b);
  void* user;
};

template <typename R>
int potrf_diag(C_t<R>* A, long lda, long sA, int batch, int j0, C_t<R>* Dinv, long sD, int* flag,
               hipStream_t st);

template <typename R>
int potrf_batched(C_t<R>* A, int n, long lda, long sA, int batch, C_t<R>* Dinv, long sD, int* flag,
                  hipStream_t st, const ProfHook* hook = nullptr);

// sbinv (may be NULL): inverses of the diagonal super-blocks from sb_inverse_batched;
// given, narrow solves (nc <= 32) run as GEMMs only, skipping the matrices whose kact
// entry is 0 (kact may be NULL), and right-hand side b uses factor fmap[b] (device
// array; NULL: factor b; non-NULL requires sbinv).  nacc (> 0): the number of
// right-hand-side blocks the timing hook counts as work (the active ones).
template <typename R>
int potrs_batched(const C_t<R>* L, int n, long lda, long sL, int batch, const C_t<R>* Dinv, long sD,
                  C_t<R>* B, long ldb, long sB, C_t<R>* Z, long ldz, long sZ, int nc, hipStream_t st,
                  const ProfHook* hook = nullptr, const C_t<R>* sbinv = nullptr, const int* kact = nullptr,
                  const int* fmap = nullptr, int nacc = 0);

// Inverses of the diagonal super-blocks (256 wide in FP32, 128 in FP64) of a batch of
// Cholesky factors: nsb = ceil(n / WS) blocks of WS x WS per matrix (ld WS); and the block
// columns below the super-blocks copied, conjugate-transposed, into the upper triangle of L
// (which the factorisation leaves unused), as the super-block solves read them.  Dinv: the
// factorisation's inverted 64 x 64 diagonal blocks; n a multiple of 64; work: device
// scratch of batch nsb (WS^2 + WS^2 / 4) elements.
template <typename R>
int sb_inverse_batched(C_t<R>* L, int n, long lda, long sL, int batch, const C_t<R>* Dinv, long sD,
                       C_t<R>* SBinv, C_t<R>* work, hipStream_t st);

}  // namespace phx
