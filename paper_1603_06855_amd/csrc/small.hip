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

// Wave-level sum and max (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
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

// Omega-orthonormalisation coefficients from the Hermitian Gram matrix in Ls (m x m,
// [col][row]), in place: columns scaled to unit norm (D), Cholesky with dropping (a pivot at
// or below `drop` drops its column: kp = 0), then the inverse Xs of the lower factor.
// Every thread of the workgroup calls it.  The factorisation takes two barriers per
// column: every thread takes the same pivot decision from the same value, the scaled
// column goes to lc, then the trailing update reads lc; the inverse needs none: lane t
// forms column t of L^{-1} by forward substitution, reading only the finished factor and
// its own column.
__device__ void chol_drop_all(double2 (&Ls)[64][65], double2 (&Xs)[64][65], double* D, int* kp, double2* lc, int m,
                              double drop) {
  const int tid = threadIdx.x;
  if (tid < m) {
    const double d = Ls[tid][tid].x;
    const bool ok = d > 1e-300 && isfinite(d);
    D[tid] = ok ? 1.0 / sqrt(d) : 0.0;
    kp[tid] = ok ? 1 : 0;
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += SMALL_NT) {
    const int i = e % m, j = e / m;
    Ls[j][i] = cscale(Ls[j][i], D[i] * D[j]);
  }
  __syncthreads();
  for (int c = 0; c < m; ++c) {
    const double pv = Ls[c][c].x;
    const int kc = kp[c] && (pv > drop);
    const double pc = kc ? sqrt(pv) : 0.0;
    if (tid < m) lc[tid] = (tid > c && pc > 0) ? cscale(Ls[c][tid], 1.0 / pc) : make_double2(0, 0);
    __syncthreads();  // every thread has read the pivot; lc complete
    if (tid == 0) kp[c] = kc;
    if (pc > 0) {
      if (tid < m) Ls[c][tid] = tid == c ? make_double2(pc, 0.0) : (tid > c ? lc[tid] : Ls[c][tid]);
      const int r = m - c - 1;  // trailing rows and columns c+1 .. m-1
      for (int e = tid; e < r * r; e += SMALL_NT) {
        const int i = c + 1 + e % r, j = c + 1 + e / r;
        if (i >= j) Ls[j][i] = csub(Ls[j][i], cmulc(lc[i], lc[j]));
      }
    } else {
      if (tid < m) Ls[c][tid] = make_double2(tid == c ? 1.0 : 0.0, 0.0);
      if (tid < c) Ls[tid][c] = make_double2(0.0, 0.0);
    }
    __syncthreads();
  }
  if (tid < m) {  // column t of L^{-1}: rows t .. m-1
    const int t = tid;
    for (int i = 0; i < t; ++i) Xs[t][i] = make_double2(0.0, 0.0);
    for (int i = t; i < m; ++i) {
      double2 sacc = make_double2(i == t ? 1.0 : 0.0, 0.0);
      for (int l = t; l < i; ++l) sacc = csub(sacc, cmul(Ls[l][i], Xs[t][l]));
      Xs[t][i] = cscale(sacc, 1.0 / Ls[i][i].x);
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(SMALL_NT) void chol_drop_kernel(const double2* G, int m, double drop, double2* C0,
                                                        int* keep, const int* kact) {
  if (kact && !kact[blockIdx.x]) return;  // a converged k-point
  __shared__ double2 Ls[64][65];  // [col][row]
  __shared__ double2 Xs[64][65];
  __shared__ double D[64];
  __shared__ int kp[64];
  __shared__ double2 lc[64];
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const double2* Gk = G + (long)k * m * m;
  for (int e = tid; e < m * m; e += SMALL_NT) {
    const int i = e % m, j = e / m;
    const double2 a = Gk[i + j * m], b = Gk[j + i * m];
    Ls[j][i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
  __syncthreads();
  chol_drop_all(Ls, Xs, D, kp, lc, m, drop);
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
                                                     int* sweeps_out, const int* kact) {
  if (kact && !kact[blockIdx.x]) return;  // a converged k-point: its Ritz values stay
  __shared__ JacobiLDS L;
  __shared__ double D[64];
  __shared__ int kp[64];
  __shared__ double2 lc[64];
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
  chol_drop_all(Ls, Xs, D, kp, lc, m, drop);
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
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * SMALL_NT;
    if (e >= mm * mm) break;
    L.As[e / mm][e % mm] = acc[q];
  }
  const double big = 1e3 * block_max(L, amax) + 1.0;
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
                   double2* Cp, double* theta, int* sweeps, hipStream_t st, const int* kact, long sCx) {
  hipLaunchKernelGGL(rr_gen_kernel, dim3(nk), dim3(SMALL_NT), 0, st, G2, m, s, drop, C0, keep, Cx, Cp,
                     sCx > 0 ? sCx : (long)m * s, theta, sweeps, kact);
}

void launch_rr_eig(const double2* G, const int* keep, int m, int s, int nk, double2* C, double* theta, int* sweeps,
                   hipStream_t st, const int* kact) {
  hipLaunchKernelGGL(rr_eig_kernel, dim3(nk), dim3(SMALL_NT), 0, st, G, keep, m, s, C, theta, sweeps, kact);
}

}  // namespace phx
