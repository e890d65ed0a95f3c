// Per-k small dense kernels of the block eigensolver (one workgroup per k-point,
// matrices of order m <= 64 held in LDS, FP64).
//
// chol_drop: Omega-orthonormalisation coefficients of a search basis from its Gram
//   matrix G = S^H Omega S.  Columns are scaled to unit Omega-norm, then a Cholesky
//   factorisation drops every column whose pivot falls below `drop` (it is nearly a
//   combination of the previous ones, or zero).  Output C0 = D L^{-H} with the
//   dropped columns set to zero, so S C0 has Omega-orthonormal kept columns.
// rr_eig: Rayleigh-Ritz on an Omega-orthonormal basis: eigen-decomposition of the
//   Hermitian G = S^H K S by cyclic parallel Jacobi (round-robin pair ordering),
//   returning the s lowest eigenpairs.  Dropped columns get a large diagonal so they
//   are never selected.  A pair (p, q) is rotated only while |a_pq| exceeds both
//   1e-15 sqrt(|a_pp a_qq|) (relative accuracy of the small eigenvalues) and
//   1e-18 of the largest kept diagonal entry (the zero modes at Gamma); a rotated
//   pair's off-diagonal entries are then set to zero exactly rather than left at
//   rounding level, so a sweep without rotations is reached and ends the loop.
// heev_tri: the s lowest eigenpairs of a Hermitian matrix of order n <= 64 by Householder
//   reduction to tridiagonal form, multisection on Sturm counts for the eigenvalues and
//   inverse iteration for the eigenvectors (one lane each), modified Gram-Schmidt across
//   them and the back-transformation through the reflectors.  Eigenvalues are accurate to
//   a small multiple of eps ||A|| in absolute terms (Jacobi: relative to each eigenvalue);
//   the sequence of dependent steps is a few hundred instead of sweeps x 63 rounds.
#include "phx_common.h"
#include "phx_physics.h"

namespace phx {

constexpr int SMALL_NT = 1024;  // threads per workgroup of the small kernels (latency bound)

// Shared state of the Jacobi eigensolver of one workgroup.
struct JacobiLDS {
  double2 As[64][65];  // [col][row]
  double2 Vs[64][65];
  int pp[32], qq[32], act[32];
  double cs_[32], sn_[32];
  double2 ph_[32];
  double wred[SMALL_NT / 64][2];  // per-wave partial results of a reduction
  int order[64];
  int rot[2];  // per sweep parity: some pair rotated
};

// v from lane (lane ^ 1), (lane ^ 2) or the mirrored lane of its 8- or 16-lane row (DPP
// quad_perm [1,0,3,2] and [2,3,0,1], row_half_mirror, row_mirror): register moves, no LDS.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over each 16-lane row of the wavefront, in every lane of the row.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // pairs
  v += dpp_d<0x4E>(v);   // quads
  v += dpp_d<0x141>(v);  // 8 lanes
  v += dpp_d<0x140>(v);  // 16 lanes
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int lane);

// Wave-level sum (64 lanes), the same value in every lane.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return (readlane_d(v, 15) + readlane_d(v, 31)) + (readlane_d(v, 47) + readlane_d(v, 63));
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Max-reduction of one value per thread over the workgroup (L: an LDS state with wred).
template <typename LDS>
__device__ double block_max(LDS& L, double v) {
  const int tid = threadIdx.x;
  v = wave_max(v);
  if ((tid & 63) == 0) L.wred[tid >> 6][0] = v;
  __syncthreads();
  double r = L.wred[0][0];
  for (int w = 1; w < SMALL_NT / 64; ++w) r = fmax(r, L.wred[w][0]);
  __syncthreads();
  return r;
}

// The double held by lane `lane` (wave-uniform) of the wavefront.
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 1/q from the hardware estimate and two Newton steps (a few ulp; q normal and non-zero).
__device__ __forceinline__ double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  double e = fma(-q, r, 1.0);
  r = fma(r, e, r);
  e = fma(-q, r, 1.0);
  return fma(r, e, r);
}

// Sum over the 32 lanes of each half of the wavefront.
__device__ __forceinline__ double half_sum(double v) {
  v = row16_sum(v);
  const double s0 = readlane_d(v, 15) + readlane_d(v, 31), s1 = readlane_d(v, 47) + readlane_d(v, 63);
  return (threadIdx.x & 32) ? s1 : s0;
}

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}

// Order of LDS accesses between the lanes of one wavefront that works alone (the other
// waves of the workgroup wait at a workgroup barrier afterwards): a compiler barrier with
// workgroup-scope fences, no hardware barrier.
#define WAVE_SYNC()                                        \
  do {                                                     \
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup"); \
    __builtin_amdgcn_wave_barrier();                       \
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); \
  } while (0)

// Cyclic Jacobi on the Hermitian mm x mm matrix L.As (mm even), accumulating the
// rotations into L.Vs; returns the number of sweeps.  Each round rotates the mm/2 disjoint
// pairs of the round-robin ordering at once: A <- J^H A J as (mm/2)^2 independent 2 x 2
// blocks (rows of pair i, columns of pair j) and V <- V J, two barriers per round.
__device__ int jacobi_sweeps(JacobiLDS& L, int mm, double floor_abs) {
  const int tid = threadIdx.x;
  const int half = mm / 2;
  int sw = 0;
  for (sw = 0; sw < 40; ++sw) {
    // stop when the off-diagonal part is at rounding level, or the last sweep rotated nothing
    double off = 0, dg = 0;
    for (int e = tid; e < mm * mm; e += SMALL_NT) {
      const int i = e % mm, j = e / mm;
      const double a2 = cabs2(L.As[j][i]);
      if (i == j) dg += a2; else off += a2;
    }
    off = wave_sum(off);
    dg = wave_sum(dg);
    if ((tid & 63) == 0) {
      L.wred[tid >> 6][0] = off;
      L.wred[tid >> 6][1] = dg;
    }
    __syncthreads();
    double to = 0, td = 0;
    for (int w = 0; w < SMALL_NT / 64; ++w) {
      to += L.wred[w][0];
      td += L.wred[w][1];
    }
    const bool stop = to <= 1e-32 * td || (sw > 0 && !L.rot[(sw - 1) & 1]);
    __syncthreads();  // wred and rot read by every thread before they change
    if (stop) break;
    if (tid == 0) L.rot[sw & 1] = 0;
    for (int r = 0; r < mm - 1; ++r) {
      // rotation of each pair from its 2 x 2 diagonal block; below the thresholds the pair's
      // off-diagonal entries are set to zero and its rotation is the identity
      if (tid < half) {
        int p, q;
        if (tid == 0) { p = r; q = mm - 1; }
        else { p = (r + tid) % (mm - 1); q = (r - tid + mm - 1) % (mm - 1); }
        const double a = L.As[p][p].x, b = L.As[q][q].x;
        const double2 c = L.As[q][p];  // row p, col q
        // |c| scaled so that its square cannot underflow into subnormals.
        const double cm = fmax(fabs(c.x), fabs(c.y));
        double ac = 0.0;
        if (cm > 0) {
          const double xr = c.x / cm, yr = c.y / cm;
          ac = cm * sqrt(xr * xr + yr * yr);
        }
        int act = 0;
        double cs = 1.0, sn = 0.0;
        double2 ph = make_double2(1.0, 0.0);
        if (!(ac > floor_abs && ac > 1e-15 * sqrt(fabs(a) * fabs(b)))) {
          L.As[q][p] = make_double2(0.0, 0.0);
          L.As[p][q] = make_double2(0.0, 0.0);
        } else {
          act = 1;
          ph = make_double2(c.x / ac, -c.y / ac);
          const double tau = (b - a) / (2.0 * ac);
          double t;
          if (fabs(tau) > 1e150) t = 0.5 / tau;
          else t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          cs = 1.0 / sqrt(1.0 + t * t);
          sn = t * cs;
          L.rot[sw & 1] = 1;
        }
        L.pp[tid] = p; L.qq[tid] = q; L.act[tid] = act;
        L.cs_[tid] = cs; L.sn_[tid] = sn; L.ph_[tid] = ph;
      }
      __syncthreads();
      // A <- J^H A J: block (i, j) holds rows p_i, q_i and columns p_j, q_j.  Columns
      // (A J): c_p' = cs c_p - sn ph c_q, c_q' = sn c_p + cs ph c_q; rows (J^H A):
      // r_p' = cs r_p - sn conj(ph) r_q, r_q' = sn r_p + cs conj(ph) r_q.
      for (int e = tid; e < half * half; e += SMALL_NT) {
        const int i = e % half, j = e / half;
        const int ai = L.act[i], aj = L.act[j];
        if (!ai && !aj) continue;
        const int p = L.pp[i], q = L.qq[i], pc = L.pp[j], qc = L.qq[j];
        double2 b00 = L.As[pc][p], b10 = L.As[pc][q], b01 = L.As[qc][p], b11 = L.As[qc][q];
        if (aj) {
          const double c = L.cs_[j], sj = L.sn_[j];
          const double2 ph = L.ph_[j];
          const double2 t0 = cmul(ph, b01), t1 = cmul(ph, b11);
          const double2 n00 = csub(cscale(b00, c), cscale(t0, sj)), n01 = cadd(cscale(b00, sj), cscale(t0, c));
          const double2 n10 = csub(cscale(b10, c), cscale(t1, sj)), n11 = cadd(cscale(b10, sj), cscale(t1, c));
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        if (ai) {
          const double c = L.cs_[i], si = L.sn_[i];
          const double2 phc = cconj(L.ph_[i]);
          const double2 t0 = cmul(phc, b10), t1 = cmul(phc, b11);
          const double2 n00 = csub(cscale(b00, c), cscale(t0, si)), n10 = cadd(cscale(b00, si), cscale(t0, c));
          const double2 n01 = csub(cscale(b01, c), cscale(t1, si)), n11 = cadd(cscale(b01, si), cscale(t1, c));
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        if (i == j) {  // the rotated diagonal block: exactly diagonal and real
          b00.y = 0.0;
          b11.y = 0.0;
          b01 = make_double2(0.0, 0.0);
          b10 = make_double2(0.0, 0.0);
        }
        L.As[pc][p] = b00; L.As[pc][q] = b10; L.As[qc][p] = b01; L.As[qc][q] = b11;
      }
      // V <- V J on the columns of the rotated pairs
      for (int e = tid; e < mm * half; e += SMALL_NT) {
        const int row = e % mm, j = e / mm;
        if (!L.act[j]) continue;
        const int p = L.pp[j], q = L.qq[j];
        const double c = L.cs_[j], sj = L.sn_[j];
        const double2 vp = L.Vs[p][row], phvq = cmul(L.ph_[j], L.Vs[q][row]);
        L.Vs[p][row] = csub(cscale(vp, c), cscale(phvq, sj));
        L.Vs[q][row] = cadd(cscale(vp, sj), cscale(phvq, c));
      }
      __syncthreads();
    }
  }
  return sw;
}

// Working storage of heev_tri (overlaid on JacobiLDS::Vs once the Jacobi storage is free).
constexpr int TRI_MAXS = 24;  // eigenpairs heev_tri returns at most
constexpr int TRI_LD = TRI_MAXS + 1;
struct TriLDS {
  double u[64][3][TRI_MAXS];  // rows of U of the pivoted LU of T - lambda_j I (j fastest); then Y
  double z[64][TRI_LD];       // eigenvectors of the real tridiagonal matrix, [row][j]
  double dd[64], ee[64], e2[64];
  double ds[64], e2s[64];  // dd / sigma and e2 / sigma^2, sigma the power of two nearest ||T||
  double2 ph[64];  // unitary diagonal scaling that makes the subdiagonal real
  double tau[64];
  double2 beta[64], vv[2][64], ww[2][64];  // reflector and update vector, by step parity
  double lam[TRI_MAXS], znrm[TRI_MAXS];
  int kpos[64];     // position of each kept column in the compacted matrix (-1: not in it)
  int nullidx[64];  // kept columns whose row of A' is exactly zero (deflated: eigenvalue 0)
  int ord[TRI_MAXS];     // the s lowest pairs: >= 0 heev_tri's pair, < 0 null column -ord-1
  double val[TRI_MAXS];
  int nkeep, nnull;
};
static_assert(sizeof(TriLDS) <= sizeof(double2) * 64 * 65, "TriLDS overlays JacobiLDS::Vs");

// Y[j][row]: the complex eigenvectors heev_tri returns, over the U storage.
__device__ __forceinline__ double2 (*tri_y(TriLDS& T))[64] { return reinterpret_cast<double2 (*)[64]>(&T.u[0][0][0]); }

// Number of eigenvalues of the real symmetric tridiagonal matrix below x sigma (ds, e2s: the
// matrix scaled by 1/sigma): the sign changes of the leading principal minors p_i of
// T / sigma - x I, p_0 = 1, p_1 = d_0 - x, p_{i+1} = (d_i - x) p_i - e_{i-1}^2 p_{i-1} (Sturm
// sequence).  With ||T / sigma|| < 2 a minor grows by at most 8 per row; the pair
// (p_i, p_{i-1}) is rescaled by a power of two every eight rows, which changes no sign, and
// a zero minor takes the sign opposite to its predecessor.  One FMA per row lies on the
// dependent chain.
__device__ __forceinline__ int sturm_count(const TriLDS& T, int n, double x) {
  double p1 = T.ds[0] - x, p0 = 1.0;
  if (p1 == 0.0) p1 = -1e-300;
  int c = p1 < 0.0;
#pragma unroll 8
  for (int i = 1; i < n; ++i) {
    double p = fma(T.ds[i] - x, p1, -T.e2s[i - 1] * p0);
    if (p == 0.0) p = p1 < 0.0 ? 1e-300 : -1e-300;
    c += (p < 0.0) != (p1 < 0.0);
    p0 = p1;
    p1 = p;
    if ((i & 7) == 0) {
      const int e = ilogb(fmax(fabs(p0), fabs(p1)));
      p0 = ldexp(p0, -e);
      p1 = ldexp(p1, -e);
    }
  }
  return c;
}

// A uniform value in [-1, 1) from (row, vector): the start vectors of inverse iteration.
__device__ __forceinline__ double start_entry(int t, int j) {
  unsigned h = (unsigned)(t * 73856093) ^ (unsigned)(j * 19349663 + 0x9e3779b9u);
  h ^= h >> 16;
  h *= 0x7feb352dU;
  h ^= h >> 15;
  h *= 0x846ca68bU;
  h ^= h >> 16;
  return (double)h * (2.0 / 4294967296.0) - 1.0;
}

// The s (<= TRI_MAXS, <= n) lowest eigenpairs of the Hermitian n x n matrix in A (n <= 64,
// [col][row]; overwritten by the reflectors).  Out: T.lam[0..s) ascending and the
// orthonormal eigenvectors tri_y(T)[j][0..n).  Every thread of the workgroup calls it;
// returns the largest number of multisection steps.
//   1. Householder reduction Q^H A Q = T_c (H_k = I - tau_k v_k v_k^H acting below row k),
//      one workgroup barrier pair per column; wave 0 forms v, p = tau A v and
//      w = p - (tau/2)(v^H p) v, every thread takes part in A <- A - v w^H - w v^H.
//   2. D^H T_c D = T real with non-negative off-diagonal (ph_{k+1} = ph_k beta_k/|beta_k|).
//   3. Eigenvalue j by multisection in wave j % 16: the 64 lanes evaluate Sturm counts at
//      64 interior points of the bracket, which shrinks 65-fold per step, to
//      2 eps max(|lo|, |hi|) + eps ||T||.
//   4. Eigenvector j in lane j of wave 0: two steps of inverse iteration, each solving
//      (T - lambda_j I) x = b by Gaussian elimination with partial pivoting (pivots at least
//      eps ||T|| in magnitude), from a fixed pseudo-random start; the members of a tight
//      cluster in turn, orthogonalised against the cluster's earlier vectors.
//   5. Modified Gram-Schmidt over the vectors in ascending order (it separates the vectors
//      of equal or nearly equal eigenvalues; it leaves well separated ones unchanged to
//      rounding), then y_j = Q D z_j.
__device__ __attribute__((noinline)) int heev_tri(double2 (&A)[64][65], TriLDS& T, int n, int s) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double eps = 2.220446049250313e-16;
  // 1. tridiagonalisation.  Step k: every thread applies the update of step k-1 to its
  //    entries (row i = tid % 64, columns j > k with j = k + 1 + tid / 64 mod 16) of the
  //    trailing block and adds their products with v_k to its partial sum of A_k v_k; wave 0
  //    then sums the 16 partials, forms w_k, applies both updates to column k+1 itself and
  //    builds the reflector v_{k+1} from it.  Two barriers per column.
  double2(*pp)[64] = reinterpret_cast<double2(*)[64]>(&T.u[0][0][0]);  // partial products [chunk][row]
  // Householder vector of the column held by the lanes (x in lane t > c, t < n): H x = beta e_{c+1}
  auto reflect = [&](double2 x, int c, double2& v, double& tk, double2& bk) {
    const int t = lane;
    const bool in = t > c && t < n;
    const double a2 = wave_sum(in ? cabs2(x) : 0.0);
    const double2 x0 = make_double2(readlane_d(x.x, c + 1), readlane_d(x.y, c + 1));
    const double ax0 = sqrt(cabs2(x0));
    tk = 0.0;
    bk = x0;
    v = make_double2(0, 0);
    if (a2 - ax0 * ax0 > 0.0) {  // the same decision in every lane
      const double al = sqrt(a2);
      const double2 phs = ax0 > 0 ? make_double2(x0.x / ax0, x0.y / ax0) : make_double2(1.0, 0.0);
      bk = make_double2(-phs.x * al, -phs.y * al);
      tk = 1.0 / (al * (al + ax0));
      v = in ? ((t == c + 1) ? csub(x0, bk) : x) : make_double2(0, 0);
    }
  };
  if (n >= 3 && wave == 0) {
    double2 v;
    double tk;
    double2 bk;
    const double2 x = (lane > 0 && lane < n) ? A[0][lane] : make_double2(0, 0);
    reflect(x, 0, v, tk, bk);
    T.vv[0][lane] = v;
    if (tk != 0.0 && lane > 0 && lane < n) A[0][lane] = v;
    if (lane == 0) {
      T.tau[0] = tk;
      T.beta[0] = bk;
    }
  }
  __syncthreads();
  for (int k = 0; k + 2 < n; ++k) {
    const int cur = k & 1, prv = cur ^ 1;
    const double tk = T.tau[k];
    // phase A: deferred update of step k-1 and partial products with v_k
    {
      const int i = lane, c = wave;
      double2 part = make_double2(0, 0);
      if (i > k && i < n) {
        const double2 vi = T.vv[prv][i], wi = T.ww[prv][i];
        for (int j = k + 1 + c; j < n; j += SMALL_NT / 64) {
          double2 a = A[j][i];
          if (k > 0 && T.tau[k - 1] != 0.0) {
            a = csub(a, cadd(cmulc(vi, T.ww[prv][j]), cmulc(wi, T.vv[prv][j])));
            A[j][i] = a;
          }
          part = cadd(part, cmul(a, T.vv[cur][j]));
        }
      }
      pp[c][i] = part;
    }
    __syncthreads();
    // phase B: w_k, column k+1 of A_{k+1}, the next reflector
    if (wave == 0) {
      const int t = lane;
      const bool in = t > k && t < n;
      const double2 v = T.vv[cur][t];
      double2 w = make_double2(0, 0);
      if (tk != 0.0) {
        double2 p = make_double2(0, 0);
        if (in)
          for (int c = 0; c < SMALL_NT / 64; ++c) p = cadd(p, pp[c][t]);
        p = cscale(p, tk);
        const double vp = wave_sum(in ? v.x * p.x + v.y * p.y : 0.0);  // Re(v^H p)
        w = in ? csub(p, cscale(v, 0.5 * tk * vp)) : make_double2(0, 0);
      }
      T.ww[cur][t] = w;
      // columns k+1 (and, after the last reflector, k+2) of A_{k+1}, rows from the diagonal
      const int clast = (k + 3 < n) ? k + 1 : n - 1;
      for (int c = k + 1; c <= clast; ++c) {
        const double2 vc = make_double2(readlane_d(v.x, c), readlane_d(v.y, c));
        const double2 wc = make_double2(readlane_d(w.x, c), readlane_d(w.y, c));
        if (t >= c && t < n) {
          double2 a = A[c][t];
          if (tk != 0.0) a = csub(a, cadd(cmulc(v, wc), cmulc(w, vc)));
          A[c][t] = a;
        }
      }
      WAVE_SYNC();
      if (k + 3 < n) {  // reflector of column k+1
        double2 vn;
        double tn;
        double2 bn;
        const double2 x = (t > k + 1 && t < n) ? A[k + 1][t] : make_double2(0, 0);
        reflect(x, k + 1, vn, tn, bn);
        T.vv[prv][t] = vn;
        if (tn != 0.0 && t > k + 1 && t < n) A[k + 1][t] = vn;
        if (t == 0) {
          T.tau[k + 1] = tn;
          T.beta[k + 1] = bn;
        }
      }
    }
    __syncthreads();
  }
  // 2. the real tridiagonal matrix and the phases
  if (wave == 0) {
    const int t = lane;
    if (t < n) T.dd[t] = A[t][t].x;
    if (t == 0 && n >= 2) T.beta[n - 2] = A[n - 2][n - 1];
    WAVE_SYNC();
    double2 u = make_double2(1.0, 0.0);  // beta_t / |beta_t|
    if (t + 1 < n) {
      const double2 bt = T.beta[t];
      const double b = sqrt(cabs2(bt));
      T.ee[t] = b;
      T.e2[t] = b * b;
      if (b > 0) u = make_double2(bt.x / b, bt.y / b);
    } else if (t < 64) {
      T.ee[t] = 0.0;
      T.e2[t] = 0.0;
    }
    T.vv[0][t] = u;
    WAVE_SYNC();
    if (t == 0) {
      double2 ph = make_double2(1.0, 0.0);
      T.ph[0] = ph;
      for (int k = 0; k + 1 < n; ++k) {
        ph = cmul(ph, T.vv[0][k]);
        T.ph[k + 1] = ph;
      }
    }
  }
  __syncthreads();
  // Gershgorin bracket of the spectrum (every wave computes the same values)
  double gl, gu, emax2;
  {
    const int t = lane;
    const double d = t < n ? T.dd[t] : 0.0;
    const double r = t < n ? (t > 0 ? T.ee[t - 1] : 0.0) + T.ee[t] : 0.0;
    gl = wave_min(t < n ? d - r : 1e308);
    gu = wave_max(t < n ? d + r : -1e308);
    emax2 = wave_max(t < n ? T.e2[t] : 0.0);
  }
  const double tnorm = fmax(fabs(gl), fabs(gu));
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  const double atol = eps * tnorm + pivmin;
  const double sigma = tnorm > 0 ? ldexp(1.0, ilogb(tnorm)) : 1.0, isig = 1.0 / sigma;
  if (wave == 0 && lane < n) {
    T.ds[lane] = T.dd[lane] * isig;
    T.e2s[lane] = T.e2[lane] * isig * isig;
  }
  __syncthreads();
  gl -= 2.0 * atol;
  gu += 2.0 * atol;
  // 3. multisection: eigenvalue j = 2 w + h in half h of wave w, 32 points per step
  int steps = 0;
  {
    const int h = lane >> 5, hl = lane & 31, j = 2 * wave + h;
    double lo = gl, hi = gu;
    int it = 0;
    for (; it < 64; ++it) {
      const bool done = j >= s || hi - lo <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + atol;
      if (__ballot(!done) == 0) break;
      const double x = lo + (hi - lo) * ((hl + 1) / 33.0);
      const int c = done ? 0 : sturm_count(T, n, x * isig);
      const unsigned hm = (unsigned)(__ballot(c > j) >> (32 * h));
      const int l = hm ? __ffs(hm) - 1 : 31;
      const double xl = __shfl(x, 32 * h + l), xm = __shfl(x, 32 * h + (l > 0 ? l - 1 : 0));
      if (!done) {
        if (hm == 0) lo = xl;
        else {
          if (l > 0) lo = xm;
          hi = xl;
        }
      }
    }
    steps = it;
    // a value within the bracket's absolute resolution of zero is zero (the rigid-body
    // modes at Gamma)
    const double lm = 0.5 * (lo + hi);
    if (hl == 0 && j < s) T.lam[j] = fabs(lm) <= 4.0 * atol ? 0.0 : lm;
  }
  __syncthreads();
  // 4. inverse iteration.  Eigenvalues within ctol of their predecessor form a tight
  //    cluster (exact or near degeneracies, the zero modes at Gamma); shifts that close would
  //    all converge to the same vector, so the lanes of a cluster take their turns, each
  //    iterate orthogonalised against the cluster's earlier vectors (as LAPACK's dstein
  //    does); lanes of different clusters run together.
  if (wave == 0) {
    const int j = lane;
    const double ctol = 1e4 * atol;
    int pos = 0;
    if (j < s)
      for (int i = j; i > 0 && T.lam[i] - T.lam[i - 1] <= ctol; --i) ++pos;
    const int first = j - pos;
    const int npos = (int)wave_max(j < s ? (double)pos : 0.0);
    const double lam = j < s ? T.lam[j] : 0.0;
    const double tiny = eps * tnorm > 0 ? eps * tnorm : 2.2250738585072014e-308;
    if (j < s)
      for (int t = 0; t < n; ++t) T.z[t][j] = start_entry(t, j);
    for (int round = 0; round <= npos; ++round) {
      if (j < s && pos == round) {
        for (int rep = 0; rep < 2; ++rep) {
          // eliminate: the active row holds (a, b1) in columns (k, k+1) and right-hand side bk
          double a = T.dd[0] - lam, b1 = T.ee[0], bk = T.z[0][j];
          for (int k = 0; k + 1 < n; ++k) {
            const double e = T.ee[k], dn = T.dd[k + 1] - lam, en = T.ee[k + 1], bn = T.z[k + 1][j];
            double u0, u1, u2, rk;
            if (fabs(a) >= fabs(e)) {  // keep the active row
              if (fabs(a) < tiny) a = a < 0 ? -tiny : tiny;
              const double l = e * rcp_nr(a);
              u0 = a; u1 = b1; u2 = 0.0; rk = bk;
              a = dn - l * b1;
              b1 = en;
              bk = bn - l * bk;
            } else {  // the next row is the pivot row
              const double l = a * rcp_nr(e);
              u0 = e; u1 = dn; u2 = en; rk = bn;
              a = b1 - l * dn;
              b1 = -l * en;
              bk = bk - l * bn;
            }
            T.u[k][0][j] = rcp_nr(u0);
            T.u[k][1][j] = u1;
            T.u[k][2][j] = u2;
            T.z[k][j] = rk;
          }
          if (fabs(a) < tiny) a = a < 0 ? -tiny : tiny;
          T.u[n - 1][0][j] = rcp_nr(a);
          T.z[n - 1][j] = bk;
          // back substitution
          double x1 = 0.0, x2 = 0.0;
          for (int k = n - 1; k >= 0; --k) {
            const double x = (T.z[k][j] - T.u[k][1][j] * x1 - T.u[k][2][j] * x2) * T.u[k][0][j];
            T.z[k][j] = x;
            x2 = x1;
            x1 = x;
          }
          // orthogonal to the cluster's earlier vectors, then unit max norm
          for (int i = first; i < j; ++i) {
            double zz = 0.0, zi2 = 0.0;
            for (int t = 0; t < n; ++t) {
              zz += T.z[t][j] * T.z[t][i];
              zi2 += T.z[t][i] * T.z[t][i];
            }
            const double f = zi2 > 0 ? zz / zi2 : 0.0;
            for (int t = 0; t < n; ++t) T.z[t][j] -= f * T.z[t][i];
          }
          double xm = 0.0;
          for (int t = 0; t < n; ++t) xm = fmax(xm, fabs(T.z[t][j]));
          const double sc = xm > 0 ? 1.0 / xm : 1.0;
          for (int t = 0; t < n; ++t) T.z[t][j] *= sc;
        }
      }
      WAVE_SYNC();
    }
  }
  __syncthreads();
  // 5. modified Gram-Schmidt (vector j removed from every later vector; wave w takes the
  //    later vectors i = j + 1 + w, j + 17 + w, ..)
  for (int j = 0; j < s; ++j) {
    const double zj = lane < n ? T.z[lane][j] : 0.0;
    const double nj = wave_sum(zj * zj);
    for (int i = j + 1 + wave; i < s; i += SMALL_NT / 64) {
      const double zi = lane < n ? T.z[lane][i] : 0.0;
      const double d = nj > 0 ? wave_sum(zj * zi) / nj : 0.0;
      if (lane < n) T.z[lane][i] = zi - d * zj;
    }
    if (wave == 0 && lane == 0) T.znrm[j] = nj > 0 ? 1.0 / sqrt(nj) : 0.0;
    __syncthreads();
  }
  // back-transformation y_j = H_0 .. H_{n-3} D z_j, one half-wave per vector (rows hl and
  // hl + 32 in lane hl)
  double2(*Y)[64] = tri_y(T);
  {
    const int h = lane >> 5, hl = lane & 31, j = 2 * wave + h;
    const int t0 = hl, t1 = hl + 32;
    if (j < s) {
      const double zn = T.znrm[j];
      double2 y0 = t0 < n ? cscale(T.ph[t0], T.z[t0][j] * zn) : make_double2(0, 0);
      double2 y1 = t1 < n ? cscale(T.ph[t1], T.z[t1][j] * zn) : make_double2(0, 0);
      for (int k = n - 3; k >= 0; --k) {
        const double tk = T.tau[k];
        if (tk == 0.0) continue;
        const bool in0 = t0 > k && t0 < n, in1 = t1 > k && t1 < n;
        const double2 v0 = in0 ? A[k][t0] : make_double2(0, 0), v1 = in1 ? A[k][t1] : make_double2(0, 0);
        // v^H y
        const double dr = half_sum(v0.x * y0.x + v0.y * y0.y + v1.x * y1.x + v1.y * y1.y);
        const double di = half_sum(v0.x * y0.y - v0.y * y0.x + v1.x * y1.y - v1.y * y1.x);
        const double2 f = make_double2(tk * dr, tk * di);
        if (in0) y0 = csub(y0, cmul(v0, f));
        if (in1) y1 = csub(y1, cmul(v1, f));
      }
      Y[j][t0] = y0;
      Y[j][t1] = y1;
    }
  }
  __syncthreads();
  return steps;
}

// Omega-orthonormalisation coefficients from the Hermitian Gram matrix in Ls (m x m,
// [col][row]), in place: columns scaled to unit norm (D), Cholesky with dropping (a pivot at
// or below `drop` drops its column: kp = 0, and its row and column of the factor become
// those of the identity), and the inverse Xs of the lower factor ([col][row]).  Every thread
// of the workgroup calls it.  Blocked by panels of four columns, two barriers per panel:
// wave 0 factors the panel in registers (lane = row; the pivot decisions are taken from the
// same values in every lane) and solves its four rows of L X = I; then every thread takes
// part in the rank-4 update of the trailing lower triangle, the matching update of the rows
// of X below the panel, and the zeroing of a dropped row in earlier columns.
__device__ void chol_drop_all(double2 (&Ls)[64][65], double2 (&Xs)[64][65], double* D, int* kp, int m,
                              double drop) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid < m) {
    const double d = Ls[tid][tid].x;
    const bool ok = d > 1e-300 && isfinite(d);
    D[tid] = ok ? 1.0 / sqrt(d) : 0.0;
    kp[tid] = ok ? 1 : 0;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += SMALL_NT) {
    const int i = e & 63, j = e >> 6;
    if (i < m && j < m) Ls[j][i] = cscale(Ls[j][i], D[i] * D[j]);
    Xs[j][i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int c0 = 0; c0 < m; c0 += 4) {
    const int nq = min(4, m - c0), cb = c0 + nq;
    if (wave == 0) {
      const int t = lane;
      double2 P[4];
      double piv[4];
      int kq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) P[q] = (q < nq && t >= c0 + q && t < m) ? Ls[c0 + q][t] : make_double2(0, 0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        kq[q] = 0;
        piv[q] = 1.0;
        if (q >= nq) continue;
        const int c = c0 + q;
        const double pv = readlane_d(P[q].x, c);
        const int kc = kp[c] && pv > drop;
        kq[q] = kc;
        if (kc) {
          const double pc = sqrt(pv), ip = 1.0 / pc;
          piv[q] = pc;
          P[q] = t == c ? make_double2(pc, 0.0) : (t > c ? cscale(P[q], ip) : make_double2(0, 0));
#pragma unroll
          for (int q2 = q + 1; q2 < 4; ++q2) {
            if (q2 >= nq) continue;
            const int c2 = c0 + q2;
            const double2 l2 = make_double2(readlane_d(P[q].x, c2), readlane_d(P[q].y, c2));
            if (t >= c2) P[q2] = csub(P[q2], cmulc(P[q], l2));  // l_t conj(l_c2)
          }
        } else {
          P[q] = make_double2(t == c ? 1.0 : 0.0, 0.0);
#pragma unroll
          for (int q1 = 0; q1 < q; ++q1)
            if (t == c) P[q1] = make_double2(0, 0);  // row c of the panel's earlier columns
        }
      }
      // rows c0 .. cb-1 of X (L11 x = rhs) for the columns t < cb
      double2 x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[q] = make_double2(0, 0);
        if (q >= nq) continue;
        const int c = c0 + q;
        if (!kq[q]) {
          x[q] = make_double2(t == c ? 1.0 : 0.0, 0.0);
          continue;
        }
        double2 b = t < cb ? Xs[t][c] : make_double2(0, 0);
#pragma unroll
        for (int q1 = 0; q1 < q; ++q1) {
          const double2 lq = make_double2(readlane_d(P[q1].x, c), readlane_d(P[q1].y, c));  // L[c][c0+q1]
          b = csub(b, cmul(lq, x[q1]));
        }
        x[q] = cscale(b, 1.0 / piv[q]);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q >= nq) continue;
        if (t < m) Ls[c0 + q][t] = P[q];
        if (t < cb) Xs[t][c0 + q] = x[q];
        if (t == 0) kp[c0 + q] = kq[q];
      }
    }
    __syncthreads();
    const int r = m - cb;
    for (int e = tid; e < r * r; e += SMALL_NT) {  // trailing lower triangle
      const int i = cb + e % r, j = cb + e / r;
      if (i < j) continue;
      double2 a = Ls[j][i];
      for (int q = 0; q < nq; ++q) a = csub(a, cmulc(Ls[c0 + q][i], Ls[c0 + q][j]));
      Ls[j][i] = a;
    }
    for (int e = tid; e < r * cb; e += SMALL_NT) {  // X[i][t] -= L[i][panel] X[panel][t]
      const int i = cb + e % r, t = e / r;
      double2 a = Xs[t][i];
      for (int q = 0; q < nq; ++q) a = csub(a, cmul(Ls[c0 + q][i], Xs[t][c0 + q]));
      Xs[t][i] = a;
    }
    for (int e = tid; e < c0 * nq; e += SMALL_NT) {  // a dropped row in the earlier columns
      const int t = e % c0, q = e / c0;
      if (!kp[c0 + q]) Ls[t][c0 + q] = make_double2(0, 0);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(SMALL_NT) void chol_drop_kernel(const double2* G, int m, double drop, double2* C0,
                                                        int* keep, const int* kact) {
  if (kact && !kact[blockIdx.x]) return;  // a converged k-point
  __shared__ double2 Ls[64][65];  // [col][row]
  __shared__ double2 Xs[64][65];
  __shared__ double D[64];
  __shared__ int kp[64];
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const double2* Gk = G + (long)k * m * m;
  for (int e = tid; e < m * m; e += SMALL_NT) {
    const int i = e % m, j = e / m;
    const double2 a = Gk[i + j * m], b = Gk[j + i * m];
    Ls[j][i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
  __syncthreads();
  chol_drop_all(Ls, Xs, D, kp, m, drop);
  double2* Ck = C0 + (long)k * m * m;
  for (int e = tid; e < m * m; e += SMALL_NT) {
    const int r = e % m, c = e / m;
    // C0[r][c] = D_r conj(Linv[c][r]), Linv[c][r] = Xs[r][c]
    double2 v = make_double2(0, 0);
    if (kp[c] && c >= r) v = cscale(cconj(Xs[r][c]), D[r]);
    Ck[r + c * m] = v;
  }
  if (tid < m) keep[k * m + tid] = kp[tid];
}

// L.order[0..s) = indices of the s lowest diagonal entries of L.As (ties in index order).
__device__ void select_lowest(JacobiLDS& L, int m, int s) {
  const int tid = threadIdx.x;
  if (tid < m) {
    const double d = L.As[tid][tid].x;
    int rank = 0;
    for (int i = 0; i < m; ++i) {
      const double di = L.As[i][i].x;
      rank += (di < d || (di == d && i < tid)) ? 1 : 0;
    }
    if (rank < s) L.order[rank] = tid;
  }
  __syncthreads();
}

__global__ __launch_bounds__(SMALL_NT) void rr_eig_kernel(const double2* G, const int* keep, int m, int s, double2* C,
                                                     double* theta, int* sweeps_out, const int* kact) {
  if (kact && !kact[blockIdx.x]) return;  // a converged k-point: its Ritz values stay
  __shared__ JacobiLDS L;
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const double2* Gk = G + (long)k * m * m;
  const int* kk = keep + k * m;
  const int mm = (m + 1) & ~1;
  // Hermitian part restricted to kept columns; a scale for the large diagonal.
  double amax = 0;
  for (int e = tid; e < m * m; e += SMALL_NT) amax = fmax(amax, sqrt(cabs2(Gk[e])));
  const double big = 1e3 * block_max(L, amax) + 1.0;
  // largest kept diagonal entry: the absolute floor of the rotation threshold
  double dmax = 0;
  for (int i = tid; i < m; i += SMALL_NT)
    if (kk[i]) dmax = fmax(dmax, fabs(Gk[i + i * m].x));
  const double floor_abs = 1e-18 * block_max(L, dmax) + 1e-300;
  for (int e = tid; e < mm * mm; e += SMALL_NT) {
    const int i = e % mm, j = e / mm;
    double2 v = make_double2(0, 0);
    if (i < m && j < m) {
      if (kk[i] && kk[j]) {
        const double2 a = Gk[i + j * m], b = Gk[j + i * m];
        v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
        if (i == j) v.y = 0;
      } else if (i == j) {
        v = make_double2(big * (1.0 + i * 1e-3), 0);
      }
    } else if (i == j) {
      v = make_double2(2.0 * big, 0);
    }
    L.As[j][i] = v;
    L.Vs[j][i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int sw = jacobi_sweeps(L, mm, floor_abs);
  select_lowest(L, m, s);
  if (tid == 0 && sweeps_out) sweeps_out[k] = sw;
  for (int e = tid; e < m * s; e += SMALL_NT) {
    const int r = e % m, j = e / m;
    C[(long)k * m * s + r + (long)j * m] = L.Vs[L.order[j]][r];
  }
  if (tid < s) theta[k * s + tid] = L.As[L.order[tid]][L.order[tid]].x;
}

// Rayleigh-Ritz on a basis that is only approximately Omega-orthonormal, from its two
// Gram matrices G2 = S^H [K S | Omega S] (m x 2m per k): the Omega-Cholesky with column
// scaling and dropping (as chol_drop) gives C0 with (S C0)^H Omega (S C0) = I on the kept
// columns; the Jacobi eigenpairs V, theta of C0^H G_K C0 then give the Ritz coefficients
// in the original basis, Cx = C0 V_sel, and the previous-direction coefficients
// Cp = C0[:, s:] V[s:, sel] (the part of the Ritz vectors outside the first s columns).
// C0 (m x m per k) is scratch written and read back here.
__global__ __launch_bounds__(SMALL_NT) void rr_gen_kernel(const double2* G2, int m, int s, double drop, double2* C0g,
                                                     int* keep, double2* Cx, double2* Cp, long sCx, double* theta,
                                                     int* sweeps_out, const int* kact, int method) {
  if (kact && !kact[blockIdx.x]) return;  // a converged k-point: its Ritz values stay
  __shared__ JacobiLDS L;
  __shared__ double D[64];
  __shared__ int kp[64], nz[64];
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const double2* GK = G2 + (long)k * 2 * m * m;
  const double2* GO = GK + (long)m * m;
  const int mm = (m + 1) & ~1;
  auto& Ls = L.As;  // Cholesky factor of the scaled Omega-Gram, [col][row]
  auto& Xs = L.Vs;  // its inverse
  for (int e = tid; e < m * m; e += SMALL_NT) {
    const int i = e % m, j = e / m;
    const double2 a = GO[i + j * m], b = GO[j + i * m];
    Ls[j][i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
  __syncthreads();
  chol_drop_all(Ls, Xs, D, kp, m, drop);
  // C0[r][c] = D_r conj(Linv[c][r]) (upper triangular, dropped columns zero)
  auto c0 = [&](int r, int c) -> double2 {
    return (r < m && c < m && kp[c] && c >= r) ? cscale(cconj(Xs[r][c]), D[r]) : make_double2(0, 0);
  };
  double2* C0k = C0g + (long)k * m * m;
  for (int e = tid; e < m * m; e += SMALL_NT) {
    const int r = e % m, c = e / m;
    C0k[r + c * m] = c0(r, c);
  }
  if (tid < m) keep[k * m + tid] = kp[tid];
  // G_K (Hermitian part) into As (the factor is no longer needed: C0 comes from Xs and D),
  // T = G_K C0 into As, then A' = C0^H T, made exactly Hermitian.  Each thread owns the
  // entries (i, j) = (e % mm, e / mm), e = tid + q * SMALL_NT < mm * mm (at most four),
  // and keeps them in registers across the barrier before overwriting As.
  for (int e = tid; e < mm * mm; e += SMALL_NT) {
    const int i = e % mm, j = e / mm;
    double2 v = make_double2(0, 0);
    if (i < m && j < m) {
      const double2 a = GK[i + j * m], b = GK[j + i * m];
      v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
    L.As[j][i] = v;
  }
  __syncthreads();
  double2 acc[4];
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * SMALL_NT;
    if (e >= mm * mm) break;
    const int i = e % mm, j = e / mm;
    double2 v = make_double2(0, 0);
    if (i < m && j < m && kp[j])
      for (int l = 0; l <= j; ++l) v = cadd(v, cmul(L.As[l][i], c0(l, j)));  // G_K[i][l] C0[l][j]
    acc[q] = v;
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * SMALL_NT;
    if (e >= mm * mm) break;
    L.As[e / mm][e % mm] = acc[q];  // T[i][j]
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * SMALL_NT;
    if (e >= mm * mm) break;
    const int i = e % mm, j = e / mm;
    double2 v = make_double2(0, 0);
    if (i < m && j < m && kp[i] && kp[j])
      for (int l = 0; l <= i; ++l) v = cadd(v, cmulc(L.As[j][l], c0(l, i)));  // conj(C0[l][i]) T[l][j]
    acc[q] = v;
  }
  __syncthreads();
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * SMALL_NT;
    if (e >= mm * mm) break;
    L.As[e / mm][e % mm] = acc[q];  // A'[i][j]
  }
  __syncthreads();
  double amax = 0;
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * SMALL_NT;
    if (e >= mm * mm) break;
    const int i = e % mm, j = e / mm;
    double2 v;
    if (i == j) v = make_double2(L.As[i][i].x, 0.0);
    else {
      const double2 a = L.As[j][i], b = L.As[i][j];
      v = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
    }
    acc[q] = v;
    amax = fmax(amax, sqrt(cabs2(v)));
  }
  __syncthreads();
  const double big = 1e3 * block_max(L, amax) + 1.0;
  if (method == 1) {
    // The kept rows and columns of A', compacted, through the tridiagonal solver.  A kept
    // row that is exactly zero (a null vector of K in the basis, as the rigid translations
    // at Gamma) is deflated: eigenvalue 0 with its unit vector, exactly, so that its Ritz
    // vector stays in the null space and its residual stays exactly zero.
    TriLDS& T = *reinterpret_cast<TriLDS*>(&L.Vs[0][0]);
    if (tid < 64) nz[tid] = 0;
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * SMALL_NT;
      if (e >= mm * mm) break;
      const int i = e % mm, j = e / mm;
      if (i < m && j < m && kp[i] && kp[j] && (acc[q].x != 0.0 || acc[q].y != 0.0)) nz[i] = 1;
    }
    __syncthreads();
    if (tid == 0) {
      int c = 0, z = 0;
      for (int i = 0; i < 64; ++i) {
        const bool kept = i < m && kp[i];
        T.kpos[i] = (kept && nz[i]) ? c++ : -1;
        if (kept && !nz[i]) T.nullidx[z++] = i;
      }
      T.nkeep = c;
      T.nnull = z;
    }
    __syncthreads();
    const int n = T.nkeep, sn = min(s, n);
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * SMALL_NT;
      if (e >= mm * mm) break;
      const int i = e % mm, j = e / mm;
      if (i < m && j < m && T.kpos[i] >= 0 && T.kpos[j] >= 0) L.As[T.kpos[j]][T.kpos[i]] = acc[q];
    }
    __syncthreads();
    const int st = sn > 0 ? heev_tri(L.As, T, n, sn) : 0;
    if (tid == 0) {  // the s lowest of the deflated zeros and heev_tri's values, ascending
      int a = 0, b = 0;
      for (int j = 0; j < s; ++j) {
        if (a < T.nnull && (b >= sn || 0.0 <= T.lam[b])) {
          T.ord[j] = -(a + 1);
          T.val[j] = 0.0;
          ++a;
        } else if (b < sn) {
          T.ord[j] = b;
          T.val[j] = T.lam[b];
          ++b;
        } else {
          T.ord[j] = -1000;  // fewer kept columns than wanted pairs
          T.val[j] = big * (1.0 + j * 1e-3);
        }
      }
      if (sweeps_out) sweeps_out[k] = st;
    }
    __threadfence();  // C0k written above is read back below
    __syncthreads();
    // C0 back into LDS (As, free now): C0s[c][r]
    for (int e = tid; e < m * m; e += SMALL_NT) L.As[e / m][e % m] = C0k[e];
    __syncthreads();
    const double2(*Y)[64] = tri_y(T);
    for (int e = tid; e < m * s; e += SMALL_NT) {
      const int r = e % m, j = e / m, o = T.ord[j];
      double2 x = make_double2(0, 0), pdir = make_double2(0, 0);
      if (o >= 0) {
        for (int l = r; l < m; ++l) {
          const int kl = T.kpos[l];
          if (kl < 0) continue;
          const double2 t = cmul(L.As[l][r], Y[o][kl]);
          x = cadd(x, t);
          if (l >= s) pdir = cadd(pdir, t);
        }
      } else if (o > -1000) {
        const int i = T.nullidx[-o - 1];
        x = r <= i ? L.As[i][r] : make_double2(0, 0);
        if (i >= s) pdir = x;
      }
      Cx[(long)k * sCx + r + (long)j * m] = x;
      Cp[(long)k * sCx + r + (long)j * m] = pdir;
    }
    if (tid < s) theta[k * s + tid] = T.val[tid];
    return;
  }
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * SMALL_NT;
    if (e >= mm * mm) break;
    L.As[e / mm][e % mm] = acc[q];
  }
  __syncthreads();
  double dmax = 0;
  for (int i = tid; i < m; i += SMALL_NT)
    if (kp[i]) dmax = fmax(dmax, fabs(L.As[i][i].x));
  const double floor_abs = 1e-18 * block_max(L, dmax) + 1e-300;
  for (int e = tid; e < mm * mm; e += SMALL_NT) {
    const int i = e % mm, j = e / mm;
    if (i == j) {
      if (i >= m) L.As[i][i] = make_double2(2.0 * big, 0);
      else if (!kp[i]) L.As[i][i] = make_double2(big * (1.0 + i * 1e-3), 0);
      else L.As[i][i].y = 0;
    }
    L.Vs[j][i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int sw = jacobi_sweeps(L, mm, floor_abs);
  select_lowest(L, m, s);
  if (tid == 0 && sweeps_out) sweeps_out[k] = sw;
  __threadfence();  // C0k written above is read back below
  __syncthreads();
  for (int e = tid; e < m * s; e += SMALL_NT) {
    const int r = e % m, j = e / m;
    const int o = L.order[j];
    double2 x = make_double2(0, 0), pdir = make_double2(0, 0);
    for (int l = r; l < m; ++l) {
      const double2 t = cmul(C0k[r + l * m], L.Vs[o][l]);
      x = cadd(x, t);
      if (l >= s) pdir = cadd(pdir, t);
    }
    Cx[(long)k * sCx + r + (long)j * m] = x;
    Cp[(long)k * sCx + r + (long)j * m] = pdir;
  }
  if (tid < s) theta[k * s + tid] = L.As[L.order[tid]][L.order[tid]].x;
}

void launch_chol_drop(const double2* G, int m, int nk, double drop, double2* C0, int* keep, hipStream_t st,
                      const int* kact) {
  hipLaunchKernelGGL(chol_drop_kernel, dim3(nk), dim3(SMALL_NT), 0, st, G, m, drop, C0, keep, kact);
}

void launch_rr_gen(const double2* G2, int m, int s, int nk, double drop, double2* C0, int* keep, double2* Cx,
                   double2* Cp, double* theta, int* sweeps, hipStream_t st, const int* kact, long sCx, int method) {
  if (s > TRI_MAXS) method = 0;  // the tridiagonal solver returns at most TRI_MAXS pairs
  hipLaunchKernelGGL(rr_gen_kernel, dim3(nk), dim3(SMALL_NT), 0, st, G2, m, s, drop, C0, keep, Cx, Cp,
                     sCx > 0 ? sCx : (long)m * s, theta, sweeps, kact, method);
}

void launch_rr_eig(const double2* G, const int* keep, int m, int s, int nk, double2* C, double* theta, int* sweeps,
                   hipStream_t st, const int* kact) {
  hipLaunchKernelGGL(rr_eig_kernel, dim3(nk), dim3(SMALL_NT), 0, st, G, keep, m, s, C, theta, sweeps, kact);
}

}  // namespace phx
