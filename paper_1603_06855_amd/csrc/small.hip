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

__global__ __launch_bounds__(SMALL_NT) void chol_drop_kernel(const double2* G, int m, double drop, double2* C0,
                                                        int* keep, const int* kact) {
  if (kact && !kact[blockIdx.x]) return;  // a converged k-point
  __shared__ double2 Ls[64][65];  // [col][row]
  __shared__ double2 Xs[64][65];
  __shared__ double D[64];
  __shared__ int kp[64];
  __shared__ double piv;
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const double2* Gk = G + (long)k * m * m;
  for (int e = tid; e < m * m; e += SMALL_NT) {
    const int i = e % m, j = e / m;
    const double2 a = Gk[i + j * m], b = Gk[j + i * m];
    Ls[j][i] = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  }
  __syncthreads();
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
    if (tid == 0) {
      const double pv = Ls[c][c].x;
      const int kc = kp[c] && (pv > drop);
      kp[c] = kc;
      piv = kc ? sqrt(pv) : 0.0;
    }
    __syncthreads();
    const double pc = piv;
    if (pc > 0) {
      if (tid == c) Ls[c][c] = make_double2(pc, 0.0);
      if (tid > c && tid < m) Ls[c][tid] = cscale(Ls[c][tid], 1.0 / pc);
    } else {
      if (tid < m) Ls[c][tid] = make_double2(tid == c ? 1.0 : 0.0, 0.0);
      if (tid < c) Ls[tid][c] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (pc > 0) {
      for (int e = tid; e < m * m; e += SMALL_NT) {
        const int i = e % m, j = e / m;
        if (j > c && i >= j) Ls[j][i] = csub(Ls[j][i], cmulc(Ls[c][i], Ls[c][j]));
      }
    }
    __syncthreads();
  }
  // Xs = L^{-1}, one row at a time (thread t owns column t).
  for (int i = 0; i < m; ++i) {
    if (tid < m) {
      const int t = tid;
      double2 v = make_double2(0, 0);
      if (t <= i) {
        double2 s = make_double2(t == i ? 1.0 : 0.0, 0.0);
        for (int l = t; l < i; ++l) s = csub(s, cmul(Ls[l][i], Xs[t][l]));
        v = cscale(s, 1.0 / Ls[i][i].x);
      }
      Xs[t][i] = v;
    }
    __syncthreads();
  }
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

// Shared state of the Jacobi eigensolver of one workgroup.
struct JacobiLDS {
  double2 As[64][65];  // [col][row]
  double2 Vs[64][65];
  int pp[32], qq[32];
  double cs_[32], sn_[32];
  double2 ph_[32];
  double red[SMALL_NT], red2[SMALL_NT];
  int order[64];
  int stop, rotated, nact;
};

// Max-reduction of one value per thread over the workgroup (uses L.red).
__device__ double block_max(JacobiLDS& L, double v) {
  const int tid = threadIdx.x;
  L.red[tid] = v;
  __syncthreads();
  for (int w = SMALL_NT / 2; w > 0; w >>= 1) {
    if (tid < w) L.red[tid] = fmax(L.red[tid], L.red[tid + w]);
    __syncthreads();
  }
  const double r = L.red[0];
  __syncthreads();
  return r;
}

// Cyclic Jacobi on the Hermitian mm x mm matrix L.As (mm even), accumulating the
// rotations into L.Vs; returns the number of sweeps.
__device__ int jacobi_sweeps(JacobiLDS& L, int mm, double floor_abs) {
  const int tid = threadIdx.x;
  const int half = mm / 2;
  int sw = 0;
  for (sw = 0; sw < 40; ++sw) {
    double off = 0, dg = 0;
    for (int e = tid; e < mm * mm; e += SMALL_NT) {
      const int i = e % mm, j = e / mm;
      const double a2 = cabs2(L.As[j][i]);
      if (i == j) dg += a2; else off += a2;
    }
    L.red[tid] = off;
    L.red2[tid] = dg;
    __syncthreads();
    for (int w = SMALL_NT / 2; w > 0; w >>= 1) {
      if (tid < w) {
        L.red[tid] += L.red[tid + w];
        L.red2[tid] += L.red2[tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      L.stop = (L.red[0] <= 1e-32 * L.red2[0] || (sw > 0 && !L.rotated)) ? 1 : 0;
      L.rotated = 0;
    }
    __syncthreads();
    if (L.stop) break;
    for (int r = 0; r < mm - 1; ++r) {
      // Pair setup (wave 0): rotations below threshold are skipped; the pairs that do
      // rotate are compacted so that the two update phases touch only their columns.
      bool act = false;
      int p = 0, q = 0;
      double cs = 1.0, sn = 0.0;
      double2 ph = make_double2(1.0, 0.0);
      if (tid < half) {
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
        if (!(ac > floor_abs && ac > 1e-15 * sqrt(fabs(a) * fabs(b)))) {
          // below the thresholds: set to zero (this pair owns both entries)
          L.As[q][p] = make_double2(0.0, 0.0);
          L.As[p][q] = make_double2(0.0, 0.0);
        } else {
          act = true;
          ph = make_double2(c.x / ac, -c.y / ac);
          const double tau = (b - a) / (2.0 * ac);
          double t;
          if (fabs(tau) > 1e150) t = 0.5 / tau;
          else t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          cs = 1.0 / sqrt(1.0 + t * t);
          sn = t * cs;
        }
      }
      if (tid < 64) {
        const unsigned long long mask = __ballot(act);
        if (act) {
          const int slot = __popcll(mask & ((1ull << tid) - 1ull));
          L.pp[slot] = p; L.qq[slot] = q; L.cs_[slot] = cs; L.sn_[slot] = sn; L.ph_[slot] = ph;
        }
        if (tid == 0) {
          L.nact = __popcll(mask);
          if (L.nact) L.rotated = 1;
        }
      }
      __syncthreads();
      const int na = L.nact;
      if (na == 0) continue;  // uniform: every thread read the same count after the barrier
      // columns: A <- A J, V <- V J
      for (int e = tid; e < na * mm; e += SMALL_NT) {
        const int i = e / mm, row = e % mm;
        const int p = L.pp[i], q = L.qq[i];
        const double cs = L.cs_[i], sn = L.sn_[i];
        const double2 ph = L.ph_[i];
        const double2 ap = L.As[p][row], aq = L.As[q][row];
        const double2 phaq = cmul(ph, aq);
        L.As[p][row] = csub(cscale(ap, cs), cscale(phaq, sn));
        L.As[q][row] = cadd(cscale(ap, sn), cscale(phaq, cs));
        const double2 vp = L.Vs[p][row], vq = L.Vs[q][row];
        const double2 phvq = cmul(ph, vq);
        L.Vs[p][row] = csub(cscale(vp, cs), cscale(phvq, sn));
        L.Vs[q][row] = cadd(cscale(vp, sn), cscale(phvq, cs));
      }
      __syncthreads();
      // rows: A <- J^H A
      for (int e = tid; e < na * mm; e += SMALL_NT) {
        const int i = e / mm, col = e % mm;
        const int p = L.pp[i], q = L.qq[i];
        const double cs = L.cs_[i], sn = L.sn_[i];
        const double2 phc = cconj(L.ph_[i]);
        const double2 ap = L.As[col][p], aq = L.As[col][q];
        const double2 phaq = cmul(phc, aq);
        L.As[col][p] = csub(cscale(ap, cs), cscale(phaq, sn));
        L.As[col][q] = cadd(cscale(ap, sn), cscale(phaq, cs));
      }
      __syncthreads();
      if (tid < na) {
        const int p = L.pp[tid], q = L.qq[tid];
        L.As[q][p] = make_double2(0.0, 0.0);
        L.As[p][q] = make_double2(0.0, 0.0);
        L.As[p][p].y = 0.0;
        L.As[q][q].y = 0.0;
      }
      __syncthreads();
    }
  }
  return sw;
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
  __shared__ double piv;
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
    if (tid == 0) {
      const double pv = Ls[c][c].x;
      const int kc = kp[c] && (pv > drop);
      kp[c] = kc;
      piv = kc ? sqrt(pv) : 0.0;
    }
    __syncthreads();
    const double pc = piv;
    if (pc > 0) {
      if (tid == c) Ls[c][c] = make_double2(pc, 0.0);
      if (tid > c && tid < m) Ls[c][tid] = cscale(Ls[c][tid], 1.0 / pc);
    } else {
      if (tid < m) Ls[c][tid] = make_double2(tid == c ? 1.0 : 0.0, 0.0);
      if (tid < c) Ls[tid][c] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (pc > 0) {
      for (int e = tid; e < m * m; e += SMALL_NT) {
        const int i = e % m, j = e / m;
        if (j > c && i >= j) Ls[j][i] = csub(Ls[j][i], cmulc(Ls[c][i], Ls[c][j]));
      }
    }
    __syncthreads();
  }
  for (int i = 0; i < m; ++i) {  // Xs = L^{-1}, one row at a time (thread t owns column t)
    if (tid < m) {
      const int t = tid;
      double2 v = make_double2(0, 0);
      if (t <= i) {
        double2 sacc = make_double2(t == i ? 1.0 : 0.0, 0.0);
        for (int l = t; l < i; ++l) sacc = csub(sacc, cmul(Ls[l][i], Xs[t][l]));
        v = cscale(sacc, 1.0 / Ls[i][i].x);
      }
      Xs[t][i] = v;
    }
    __syncthreads();
  }
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
