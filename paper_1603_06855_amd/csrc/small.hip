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
                                                        int* keep) {
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

__global__ __launch_bounds__(SMALL_NT) void rr_eig_kernel(const double2* G, const int* keep, int m, int s, double2* C,
                                                     double* theta, int* sweeps_out) {
  __shared__ double2 As[64][65];  // [col][row]
  __shared__ double2 Vs[64][65];
  __shared__ int pp[32], qq[32];
  __shared__ double cs_[32], sn_[32];
  __shared__ double2 ph_[32];
  __shared__ double red[SMALL_NT], red2[SMALL_NT];
  __shared__ int order[64];
  __shared__ int stop;
  __shared__ int rotated;
  __shared__ int nact;
  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const double2* Gk = G + (long)k * m * m;
  const int* kk = keep + k * m;
  const int mm = (m + 1) & ~1;
  // Hermitian part restricted to kept columns; a scale for the large diagonal.
  double amax = 0;
  for (int e = tid; e < m * m; e += SMALL_NT) amax = fmax(amax, sqrt(cabs2(Gk[e])));
  red[tid] = amax;
  __syncthreads();
  for (int w = SMALL_NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double big = 1e3 * red[0] + 1.0;
  __syncthreads();
  // largest kept diagonal entry: the absolute floor of the rotation threshold
  double dmax = 0;
  for (int i = tid; i < m; i += SMALL_NT)
    if (kk[i]) dmax = fmax(dmax, fabs(Gk[i + i * m].x));
  red[tid] = dmax;
  __syncthreads();
  for (int w = SMALL_NT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double floor_abs = 1e-18 * red[0] + 1e-300;
  __syncthreads();
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
    As[j][i] = v;
    Vs[j][i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  int sw = 0;
  const int half = mm / 2;
  for (sw = 0; sw < 40; ++sw) {
    double off = 0, dg = 0;
    for (int e = tid; e < mm * mm; e += SMALL_NT) {
      const int i = e % mm, j = e / mm;
      const double a2 = cabs2(As[j][i]);
      if (i == j) dg += a2; else off += a2;
    }
    red[tid] = off;
    red2[tid] = dg;
    __syncthreads();
    for (int w = SMALL_NT / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[tid] += red[tid + w];
        red2[tid] += red2[tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      stop = (red[0] <= 1e-32 * red2[0] || (sw > 0 && !rotated)) ? 1 : 0;
      rotated = 0;
    }
    __syncthreads();
    if (stop) break;
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
        const double a = As[p][p].x, b = As[q][q].x;
        const double2 c = As[q][p];  // row p, col q
        // |c| scaled so that its square cannot underflow into subnormals.
        const double cm = fmax(fabs(c.x), fabs(c.y));
        double ac = 0.0;
        if (cm > 0) {
          const double xr = c.x / cm, yr = c.y / cm;
          ac = cm * sqrt(xr * xr + yr * yr);
        }
        if (!(ac > floor_abs && ac > 1e-15 * sqrt(fabs(a) * fabs(b)))) {
          // below the thresholds: set to zero (this pair owns both entries)
          As[q][p] = make_double2(0.0, 0.0);
          As[p][q] = make_double2(0.0, 0.0);
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
          pp[slot] = p; qq[slot] = q; cs_[slot] = cs; sn_[slot] = sn; ph_[slot] = ph;
        }
        if (tid == 0) {
          nact = __popcll(mask);
          if (nact) rotated = 1;
        }
      }
      __syncthreads();
      const int na = nact;
      if (na == 0) continue;  // uniform: every thread read the same count after the barrier
      // columns: A <- A J, V <- V J
      for (int e = tid; e < na * mm; e += SMALL_NT) {
        const int i = e / mm, row = e % mm;
        const int p = pp[i], q = qq[i];
        const double cs = cs_[i], sn = sn_[i];
        const double2 ph = ph_[i];
        const double2 ap = As[p][row], aq = As[q][row];
        const double2 phaq = cmul(ph, aq);
        As[p][row] = csub(cscale(ap, cs), cscale(phaq, sn));
        As[q][row] = cadd(cscale(ap, sn), cscale(phaq, cs));
        const double2 vp = Vs[p][row], vq = Vs[q][row];
        const double2 phvq = cmul(ph, vq);
        Vs[p][row] = csub(cscale(vp, cs), cscale(phvq, sn));
        Vs[q][row] = cadd(cscale(vp, sn), cscale(phvq, cs));
      }
      __syncthreads();
      // rows: A <- J^H A
      for (int e = tid; e < na * mm; e += SMALL_NT) {
        const int i = e / mm, col = e % mm;
        const int p = pp[i], q = qq[i];
        const double cs = cs_[i], sn = sn_[i];
        const double2 phc = cconj(ph_[i]);
        const double2 ap = As[col][p], aq = As[col][q];
        const double2 phaq = cmul(phc, aq);
        As[col][p] = csub(cscale(ap, cs), cscale(phaq, sn));
        As[col][q] = cadd(cscale(ap, sn), cscale(phaq, cs));
      }
      __syncthreads();
      if (tid < na) {
        const int p = pp[tid], q = qq[tid];
        As[q][p] = make_double2(0.0, 0.0);
        As[p][q] = make_double2(0.0, 0.0);
        As[p][p].y = 0.0;
        As[q][q].y = 0.0;
      }
      __syncthreads();
    }
  }
  // selection of the s lowest diagonal entries (ties in index order): each entry's rank
  if (tid < m) {
    const double d = As[tid][tid].x;
    int rank = 0;
    for (int i = 0; i < m; ++i) {
      const double di = As[i][i].x;
      rank += (di < d || (di == d && i < tid)) ? 1 : 0;
    }
    if (rank < s) order[rank] = tid;
  }
  if (tid == 0 && sweeps_out) sweeps_out[k] = sw;
  __syncthreads();
  for (int e = tid; e < m * s; e += SMALL_NT) {
    const int r = e % m, j = e / m;
    C[(long)k * m * s + r + (long)j * m] = Vs[order[j]][r];
  }
  if (tid < s) theta[k * s + tid] = As[order[tid]][order[tid]].x;
}

void launch_chol_drop(const double2* G, int m, int nk, double drop, double2* C0, int* keep, hipStream_t st) {
  hipLaunchKernelGGL(chol_drop_kernel, dim3(nk), dim3(SMALL_NT), 0, st, G, m, drop, C0, keep);
}

void launch_rr_eig(const double2* G, const int* keep, int m, int s, int nk, double2* C, double* theta, int* sweeps,
                   hipStream_t st) {
  hipLaunchKernelGGL(rr_eig_kernel, dim3(nk), dim3(SMALL_NT), 0, st, G, keep, m, s, C, theta, sweeps);
}

}  // namespace phx
