// Method-specific kernels: material fields, centroid-rule Fourier coefficients,
// Toeplitz gathers, the k-dependent operators of the mixed eigenproblem and the
// adjoint field energies.
//
// Notation (paper, "Phononic band structure calculation" and "Vectorization and
// parallel computations"): N = (2M+1)^3 plane waves n_p, K_p = T^T (Q + n_p),
// voxel fractions s_e = (i + 1/2)/N_v.  All quantities are non-dimensional:
// lengths by the cube edge a, stresses by phase-0 Young's modulus, density by
// phase-0 density.
//
// Compliance is handled in Mandel form, D_e = c_vol,e P_vol + c_dev,e P_dev, with
// the two isotropic projectors shared by every voxel; hence the 6N x 6N matrix
// of Eq. (7) is Phi_vol (x) P_vol + Phi_dev (x) P_dev and its inverse splits the
// same way.  Displacement vectors are stored component-major: row c*Np + p.
#include <hip/hip_ext.h>

#include <cmath>

#include "phx_common.h"
#include "phx_internal.h"
#include "phx_physics.h"

namespace phx {

// exp(sgn * i 2 pi m (i + 1/2) / nv) with exact argument reduction.
__device__ __forceinline__ double2 voxel_phase(int m, int i, int nv, int sgn) {
  long t = (long)m * (2 * i + 1);
  long mod = 2L * nv;
  t %= mod;
  if (t < 0) t += mod;
  double s, c;
  sincospi((double)t / (double)nv, &s, &c);
  return make_double2(c, sgn * s);
}

// ---------------------------------------------------------------------------
// a1: per-voxel density and Mandel compliance channels, affine in w = rho^p.
// ---------------------------------------------------------------------------
__global__ void fields_kernel(const double* rho, int nvox, MaterialND mat, double* F) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nvox) return;
  const double r = rho[e];
  const double w = pow(r, mat.p);
  F[e] = mat.dens0 + w * mat.ddens;
  F[nvox + e] = mat.cvol0 + w * mat.dcvol;
  F[2 * nvox + e] = mat.cdev0 + w * mat.dcdev;
}

// ---------------------------------------------------------------------------
// a2: ghat(m) = v sum_e g_e exp(i 2 pi m . s_e), m in [-2M, 2M]^3, by three
// one-axis partial sums (exactly the centroid sum, re-associated).
// ---------------------------------------------------------------------------
__global__ void dft_pass1(const double* F, int nv, int M2, double2* G1, int nf) {
  // G1[f][i1][i2][m3]
  const int L = 2 * M2 + 1;
  const long total = (long)nf * nv * nv * L;
  const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int m3 = (int)(id % L);
  const long fi = id / L;  // f, i1, i2
  const double* src = F + fi * nv;
  double2 acc = make_double2(0, 0);
  for (int i3 = 0; i3 < nv; ++i3) {
    const double2 e = voxel_phase(m3 - M2, i3, nv, +1);
    acc.x += e.x * src[i3];
    acc.y += e.y * src[i3];
  }
  G1[id] = acc;
}

__global__ void dft_pass2(const double2* G1, int nv, int M2, double2* G2, int nf) {
  // G2[f][i1][m2][m3] = sum_i2 e(m2,i2) G1[f][i1][i2][m3]
  const int L = 2 * M2 + 1;
  const long total = (long)nf * nv * L * L;
  const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int m3 = (int)(id % L);
  const int m2 = (int)((id / L) % L);
  const long fi1 = id / ((long)L * L);
  const double2* src = G1 + fi1 * (long)nv * L + m3;
  double2 acc = make_double2(0, 0);
  for (int i2 = 0; i2 < nv; ++i2) acc = cadd(acc, cmul(voxel_phase(m2 - M2, i2, nv, +1), src[(long)i2 * L]));
  G2[id] = acc;
}

__global__ void dft_pass3(const double2* G2, int nv, int M2, double v, double2* T, int nf) {
  // T[f][m1][m2][m3] = v sum_i1 e(m1,i1) G2[f][i1][m2][m3]
  const int L = 2 * M2 + 1;
  const long LL = (long)L * L;
  const long total = (long)nf * L * LL;
  const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const long m23 = id % LL;
  const int m1 = (int)((id / LL) % L);
  const int f = (int)(id / (L * LL));
  const double2* src = G2 + (long)f * nv * LL + m23;
  double2 acc = make_double2(0, 0);
  for (int i1 = 0; i1 < nv; ++i1) acc = cadd(acc, cmul(voxel_phase(m1 - M2, i1, nv, +1), src[(long)i1 * LL]));
  T[id] = cscale(acc, v);
}

// ---------------------------------------------------------------------------
// a3: G[p, q] = ghat(n_p - n_q) for the three tables (Omega_s, Phi_vol,
// Phi_dev), Np x Np column-major, identity on the padding.
// ---------------------------------------------------------------------------
__global__ void gather_kernel(const double2* T, int M, int N, int Np, double2* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  const int f = blockIdx.z;
  if (p >= Np) return;
  double2 v;
  if (p < N && q < N) {
    const int L = 2 * M + 1, L2 = 4 * M + 1, M2 = 2 * M;
    const int a1 = p / (L * L), a2 = (p / L) % L, a3 = p % L;
    const int b1 = q / (L * L), b2 = (q / L) % L, b3 = q % L;
    const int d1 = a1 - b1 + M2, d2 = a2 - b2 + M2, d3 = a3 - b3 + M2;
    v = T[(long)f * L2 * L2 * L2 + ((long)d1 * L2 + d2) * L2 + d3];
  } else {
    v = make_double2(p == q ? 1.0 : 0.0, 0.0);
  }
  out[(long)f * Np * Np + p + (long)q * Np] = v;
}

// Dm = Pv^{-1} - Pd^{-1}, Bm = Pd^{-1} (in place on the two inverses).
__global__ void split_inverse_kernel(double2* inv_v, double2* inv_d, long n) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  inv_v[e] = csub(inv_v[e], inv_d[e]);
}

__global__ void identity_kernel(double2* X, int n, int batch) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long nn = (long)n * n;
  if (e >= nn * batch) return;
  const long r = e % nn;
  X[e] = make_double2((r % n) == (r / n) ? 1.0 : 0.0, 0.0);
}

// K_p = T^T (Q_k + n_p) for every k of a chunk; zero on the padding.
__global__ void kvec_kernel(const double* Q, Recip Tm, int M, int N, int Np, int nk, double* Kv) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (p >= Np || k >= nk) return;
  double* o = Kv + ((long)k * Np + p) * 3;
  if (p >= N) { o[0] = o[1] = o[2] = 0; return; }
  const int L = 2 * M + 1;
  const double n1 = p / (L * L) - M, n2 = (p / L) % L - M, n3 = p % L - M;
  const double x1 = Q[3 * k] + n1, x2 = Q[3 * k + 1] + n2, x3 = Q[3 * k + 2] + n3;
  for (int c = 0; c < 3; ++c) o[c] = x1 * Tm.t[0][c] + x2 * Tm.t[1][c] + x3 * Tm.t[2][c];
}

// ---------------------------------------------------------------------------
// a6: A(k) = K(k) + sigma Omega, the Schur complement of Eq. (4) in sandwich form
//   K_pq = (2 pi V)^2 [ (Dm_pq / 3) K_p K_q^T + (Bm_pq / 2)((K_p . K_q) I + K_q K_p^T) ]
// written on the lower 64x64 tiles of the 3Np x 3Np matrix for every k of the
// chunk; each tile reads Dm, Bm, Omega_s once and emits it for all k.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void assemble_kernel(const double2* Dm, const double2* Bm, const double2* Os,
                                                        const double* Kv, int N, int Np, int nk, double c2,
                                                        const double* sigma, C_t<R>* A, long sA, int full) {
  const long t = blockIdx.x;
  int ti, tj;
  const int nt = 3 * Np / 64;
  if (full) {
    ti = (int)(t % nt);
    tj = (int)(t / nt);
  } else {
    long r = (long)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    ti = (int)r;
    tj = (int)(t - r * (r + 1) / 2);
  }
  const int i = threadIdx.x & 63;
  const int row = ti * 64 + i;
  const int ci = row / Np, p = row % Np;
  const long n3 = 3L * Np;
  for (int jj = threadIdx.x >> 6; jj < 64; jj += 4) {
    const int col = tj * 64 + jj;
    const int cj = col / Np, q = col % Np;
    const bool pad = (p >= N) || (q >= N);
    double2 dm = make_double2(0, 0), bm = dm, os = dm;
    if (!pad) {
      const long o = p + (long)q * Np;
      dm = Dm[o];
      bm = Bm[o];
      os = Os[o];
    }
    for (int k = 0; k < nk; ++k) {
      double2 v;
      if (pad) {
        v = make_double2(row == col ? 1.0 : 0.0, 0.0);
      } else {
        const double* kp = Kv + ((long)k * Np + p) * 3;
        const double* kq = Kv + ((long)k * Np + q) * 3;
        const double kk = kp[0] * kq[0] + kp[1] * kq[1] + kp[2] * kq[2];
        const double a = c2 * kp[ci] * kq[cj] / 3.0;
        const double b = c2 * 0.5 * ((ci == cj ? kk : 0.0) + kq[ci] * kp[cj]);
        v.x = a * dm.x + b * bm.x;
        v.y = a * dm.y + b * bm.y;
        if (ci == cj) {
          v.x += sigma[k] * os.x;
          v.y += sigma[k] * os.y;
        }
      }
      A[(long)k * sA + row + (long)col * n3] = mk<R>((R)v.x, (R)v.y);
    }
  }
}

// ---------------------------------------------------------------------------
// Strain of a block of displacement vectors: Mandel strain coefficients
// Y = B(K_p) X_p (6 per wave) and the trace t = K_p . X_p.
// X: 3Np x ncol per k (ld ldx, k-stride sX).  Y: Np x 6 ncol per k, t: Np x ncol.
// ---------------------------------------------------------------------------
// Strain channels of one wave: Y = (K1 x1, K2 x2, K3 x3, (K3 x2 + K2 x3)/sqrt2,
// (K3 x1 + K1 x3)/sqrt2, (K2 x1 + K1 x2)/sqrt2) (Mandel) and the trace K . x.
__device__ __forceinline__ void wave_strain(const double* K, double2 x1, double2 x2, double2 x3, double2 (&y)[6],
                                            double2& t) {
  const double r2 = 0.70710678118654752440;
  y[0] = cscale(x1, K[0]);
  y[1] = cscale(x2, K[1]);
  y[2] = cscale(x3, K[2]);
  y[3] = cscale(cadd(cscale(x2, K[2]), cscale(x3, K[1])), r2);
  y[4] = cscale(cadd(cscale(x1, K[2]), cscale(x3, K[0])), r2);
  y[5] = cscale(cadd(cscale(x1, K[1]), cscale(x2, K[0])), r2);
  t = cadd(cadd(cscale(x1, K[0]), cscale(x2, K[1])), cscale(x3, K[2]));
}

// Force of one wave from its Mandel stress S = z + (t / 3)[1,1,1,0,0,0]: c2 B(K)^T S.
__device__ __forceinline__ void wave_force(const double* K, const double2 (&z)[6], double2 t, double c2,
                                           double2 (&o)[3]) {
  const double2 t3 = cscale(t, 1.0 / 3.0);
  const double2 s0 = cadd(z[0], t3), s1 = cadd(z[1], t3), s2 = cadd(z[2], t3);
  const double r2 = 0.70710678118654752440;
  o[0] = cscale(cadd(cscale(s0, K[0]), cscale(cadd(cscale(z[4], K[2]), cscale(z[5], K[1])), r2)), c2);
  o[1] = cscale(cadd(cscale(s1, K[1]), cscale(cadd(cscale(z[3], K[2]), cscale(z[5], K[0])), r2)), c2);
  o[2] = cscale(cadd(cscale(s2, K[2]), cscale(cadd(cscale(z[3], K[1]), cscale(z[4], K[0])), r2)), c2);
}

// The pairing of each wave with its opposite.  With c = (N-1)/2 and pb = N-1-p for p < c
// (the wave index is lexicographic in n, so n_pb = -n_p and n_c = 0), the unitary U has the
// columns u_p = (e_p + e_pb)/sqrt2, u_pb = i (e_p - e_pb)/sqrt2 and u_c = e_c.  A vector's
// coordinates in that basis: (v_p, v_pb) -> U^H v = ((v_p + v_pb)/sqrt2, -i (v_p - v_pb)/sqrt2);
// back: (a, b) -> U (a, b) = ((a + i b)/sqrt2, (a - i b)/sqrt2).  Every operator built from a
// real field (Omega_s, the compliance inverses) is real symmetric in it (realify_kernel).
__device__ __forceinline__ void to_pair(double2& a, double2& b) {
  const double r2 = 0.70710678118654752440;
  const double2 sm = cadd(a, b), df = csub(a, b);
  a = cscale(sm, r2);
  b = make_double2(df.y * r2, -df.x * r2);
}
__device__ __forceinline__ void from_pair(double2& a, double2& b) {
  const double r2 = 0.70710678118654752440;
  const double2 ib = make_double2(-b.y, b.x);
  const double2 u = cscale(cadd(a, ib), r2), w = cscale(csub(a, ib), r2);
  a = u;
  b = w;
}

// Strain channels of ncol displacement columns, two formats:
// pairN = 0: Mandel strain (6 channels, Np x 6 ncol per k) and trace K . x (Np x ncol per k),
// for the compliance Bm on all six channels plus Dm on the trace (the adjoint's fields).
// pairN = N > 0: everything in the paired basis (to_pair), and the strain in the orthonormal
// basis that separates the compliance's two parts: the volumetric channel
// t0 = (e11 + e22 + e33)/sqrt3 (Np x ncol per k, for Phi_vol^-1 = Dm + Bm) and five deviatoric
// channels (e11 - e22)/sqrt2, (e11 + e22 - 2 e33)/sqrt6 and the three Mandel shears
// (Np x 5 ncol per k, for Bm = Phi_dev^-1): six operator products per vector instead of
// seven.  One thread takes both waves of a pair, returns them to plane waves, forms their
// strains and pairs the channels again (padding rows from N on are taken as they are).
__device__ __forceinline__ void dev_channels(const double2 (&y)[6], double2 t, double2 (&c)[5], double2& t0) {
  const double r2 = 0.70710678118654752440, r3 = 0.57735026918962576451, r6 = 0.40824829046386301637;
  t0 = cscale(t, r3);
  c[0] = cscale(csub(y[0], y[1]), r2);
  c[1] = cscale(csub(cadd(y[0], y[1]), cscale(y[2], 2.0)), r6);
  c[2] = y[3];
  c[3] = y[4];
  c[4] = y[5];
}
__global__ void strain_kernel(const double2* X, long ldx, long sX, const double* Kv, int Np, int ncol,
                              double2* Y, double2* tr, const int* kact, int pairN, const int* cmask) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  const int c = (pairN - 1) / 2;
  // paired basis: threads for the rows 0 .. c (row p < c with its partner N-1-p) and the
  // padding rows N .. Np-1 only (launch_strain's grid)
  if (pairN > 0 && p > c) p += pairN - 1 - c;
  if (p >= Np || (kact && !kact[k]) || (cmask && !cmask[k * ncol + j])) return;
  const double2* x = X + (long)k * sX + (long)j * ldx;
  const int nch = pairN > 0 ? 5 : 6;
  double2* y = Y + (long)k * Np * nch * ncol + (long)(nch * j) * Np;
  double2* tp = tr + (long)k * Np * ncol + (long)j * Np;
  double2 ya[6], ta;
  if (pairN == 0) {
    wave_strain(Kv + ((long)k * Np + p) * 3, x[p], x[Np + p], x[2 * Np + p], ya, ta);
    for (int ch = 0; ch < 6; ++ch) y[ch * Np + p] = ya[ch];
    tp[p] = ta;
    return;
  }
  double2 ca[5], t0a;
  if (p >= pairN || p == c) {
    wave_strain(Kv + ((long)k * Np + p) * 3, x[p], x[Np + p], x[2 * Np + p], ya, ta);
    dev_channels(ya, ta, ca, t0a);
    for (int ch = 0; ch < 5; ++ch) y[ch * Np + p] = ca[ch];
    tp[p] = t0a;
    return;
  }
  const int pb = pairN - 1 - p;
  double2 xa[3], xb[3];
  for (int d = 0; d < 3; ++d) {
    xa[d] = x[d * Np + p];
    xb[d] = x[d * Np + pb];
    from_pair(xa[d], xb[d]);
  }
  double2 yb[6], tb, cb[5], t0b;
  wave_strain(Kv + ((long)k * Np + p) * 3, xa[0], xa[1], xa[2], ya, ta);
  wave_strain(Kv + ((long)k * Np + pb) * 3, xb[0], xb[1], xb[2], yb, tb);
  dev_channels(ya, ta, ca, t0a);
  dev_channels(yb, tb, cb, t0b);
  for (int ch = 0; ch < 5; ++ch) {
    to_pair(ca[ch], cb[ch]);
    y[ch * Np + p] = ca[ch];
    y[ch * Np + pb] = cb[ch];
  }
  to_pair(t0a, t0b);
  tp[p] = t0a;
  tp[pb] = t0b;
}

// The force (2 pi V)^2 B(K_p)^T S_p of the stress in the paired basis and the channel format
// of strain_kernel's pairN > 0: Zy holds the five deviatoric channels (Bm times the strain
// channels, Np x 5 ncol per k) and Zt the volumetric one (Np x ncol per k); the Mandel
// stress is S_diag = z0 u0 + z1 u1 + z2 u2 (u0 = (1,1,1)/sqrt3, u1 = (1,-1,0)/sqrt2,
// u2 = (1,1,-2)/sqrt6) and the three shears.  KX: 3Np x ncol per k (ld ldk, k-stride sK),
// paired basis.  One thread takes both waves of a pair (p < c); padding rows from N on,
// and the centre, alone.  cmask (optional, per k * ncol + j): columns whose entry is 0 are
// skipped (strain_kernel takes the same mask).
__device__ __forceinline__ void force_of(const double* K, const double2 (&z)[5], double2 zt, double c2,
                                         double2 (&o)[3]) {
  const double r2 = 0.70710678118654752440, r3 = 0.57735026918962576451, r6 = 0.40824829046386301637;
  const double2 v = cscale(zt, r3), a = cscale(z[0], r2), b = cscale(z[1], r6);
  double2 S[6];
  S[0] = cadd(cadd(v, a), b);
  S[1] = cadd(csub(v, a), b);
  S[2] = csub(v, cscale(b, 2.0));
  S[3] = z[2];
  S[4] = z[3];
  S[5] = z[4];
  const double2 zero = make_double2(0, 0);
  wave_force(K, S, zero, c2, o);
}

__global__ void force_kernel(const double2* Zy, const double2* Zt, const double* Kv, int Np, int ncol, double c2,
                             double2* KX, long ldk, long sK, const int* kact, int pairN, const int* cmask) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  const int c = (pairN - 1) / 2;
  // threads for the rows 0 .. c (row p < c with its partner N-1-p) and the padding rows
  // N .. Np-1 only (launch_force's grid)
  if (p > c) p += pairN - 1 - c;
  if (p >= Np || (kact && !kact[k]) || (cmask && !cmask[k * ncol + j])) return;
  const double2* z = Zy + (long)k * Np * 5 * ncol + (long)(5 * j) * Np;
  const double2* zt = Zt + (long)k * Np * ncol + (long)j * Np;
  double2* o = KX + (long)k * sK + (long)j * ldk;
  double2 za[5], fa[3];
  for (int ch = 0; ch < 5; ++ch) za[ch] = z[ch * Np + p];
  if (p >= pairN || p == c) {
    force_of(Kv + ((long)k * Np + p) * 3, za, zt[p], c2, fa);
    for (int d = 0; d < 3; ++d) o[d * Np + p] = fa[d];
    return;
  }
  const int pb = pairN - 1 - p;
  double2 zb[5], fb[3];
  for (int ch = 0; ch < 5; ++ch) {
    zb[ch] = z[ch * Np + pb];
    from_pair(za[ch], zb[ch]);
  }
  double2 ta = zt[p], tb = zt[pb];
  from_pair(ta, tb);
  force_of(Kv + ((long)k * Np + p) * 3, za, ta, c2, fa);
  force_of(Kv + ((long)k * Np + pb) * 3, zb, tb, c2, fb);
  for (int d = 0; d < 3; ++d) {
    to_pair(fa[d], fb[d]);
    o[d * Np + p] = fa[d];
    o[d * Np + pb] = fb[d];
  }
}

// The Hermitian Np x Np operator Mc with Mc[N-1-p][N-1-q] = conj(Mc[p][q]) (the Fourier
// matrix of a real field on the waves n_p, n_{N-1-p} = -n_p, or its inverse) in the basis
// u_p = (e_p + e_pb)/sqrt2, u_pb = i (e_p - e_pb)/sqrt2 (p < c = (N-1)/2, pb = N-1-p),
// u_c = e_c, where it is real symmetric: Mr[a][b] = Re(u_a^H Mc u_b) (the imaginary part is
// rounding).  Rows and columns from N on (the padding) are copied.  Column-major.  Mc2
// (optional): the same for Mc + Mc2.
__global__ void realify_kernel(const double2* Mc, const double2* Mc2, int N, int Np, double* Mr) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)Np * Np) return;
  const int a = (int)(e % Np), b = (int)(e / Np);
  if (a >= N || b >= N) {
    Mr[e] = Mc[e].x + (Mc2 ? Mc2[e].x : 0.0);
    return;
  }
  const int c = (N - 1) / 2;
  const double r2 = 0.70710678118654752440;
  // u_x = al e_px + be e_qx
  auto basis = [&](int x, int& px, int& qx, double2& al, double2& be) {
    if (x == c) { px = qx = c; al = make_double2(1, 0); be = make_double2(0, 0); }
    else if (x < c) { px = x; qx = N - 1 - x; al = make_double2(r2, 0); be = make_double2(r2, 0); }
    else { px = N - 1 - x; qx = x; al = make_double2(0, r2); be = make_double2(0, -r2); }
  };
  int pa, qa, pb, qb;
  double2 aa, ba, ab, bb;
  basis(a, pa, qa, aa, ba);
  basis(b, pb, qb, ab, bb);
  auto m = [&](int r, int col) {
    const long i = r + (long)col * Np;
    return Mc2 ? cadd(Mc[i], Mc2[i]) : Mc[i];
  };
  double2 v = cmul(cmulc(ab, aa), m(pa, pb));  // conj(al_a) al_b M[pa][pb]
  if (qb != pb) v = cadd(v, cmul(cmulc(bb, aa), m(pa, qb)));
  if (qa != pa) v = cadd(v, cmul(cmulc(ab, ba), m(qa, pb)));
  if (qa != pa && qb != pb) v = cadd(v, cmul(cmulc(bb, ba), m(qa, qb)));
  Mr[e] = v.x;
}

// ---------------------------------------------------------------------------
// Eigensolver helpers.
// ---------------------------------------------------------------------------
__global__ void zero_kernel(double2* X, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    X[e] = make_double2(0, 0);
}

// Unit columns: column j of k-point k is the plane wave row idx[k s + j] (component d =
// row / Np, wave q = row % Np).  pairN = N > 0: written in the paired basis (to_pair): e_q
// with q < c has the coordinates 1/sqrt2 at q and -i/sqrt2 at N-1-q, with q > c 1/sqrt2 at
// N-1-q and i/sqrt2 at q; e_c is u_c.  The columns must be zero before.
__global__ void unit_columns_kernel(double2* X, long ldx, long sX, const int* idx, int s, int Np, int pairN) {
  const int j = threadIdx.x;
  const int k = blockIdx.x;
  if (j >= s) return;
  const int row = idx[k * s + j], q = row % Np, base = row - q;
  double2* x = X + (long)k * sX + (long)j * ldx + base;
  const int c = (pairN - 1) / 2;
  if (pairN == 0 || q >= pairN || q == c) {
    x[q] = make_double2(1.0, 0.0);
    return;
  }
  const double r2 = 0.70710678118654752440;
  const int qb = pairN - 1 - q;
  if (q < c) {
    x[q] = make_double2(r2, 0.0);
    x[qb] = make_double2(0.0, -r2);
  } else {
    x[qb] = make_double2(r2, 0.0);
    x[q] = make_double2(0.0, r2);
  }
}

// R = KX - theta OX per column (one block per (column, k)); writes R into Rp in the
// preconditioner precision, the residual norm and the relative residual
// rn = |R| / ((|theta| + sigma) |OX|).  Columns with rn below act_tol (columns from nlock
// on: below guard_tol) are locked: their residual, their previous-direction (P) column
// with its images and the images of their search direction (W) are zeroed.
template <typename R>
__global__ __launch_bounds__(256) void residual_kernel(double2* Big, long n3, long mcols, long sBig,
                                                       const double* theta, int s, const double* sigma,
                                                       double act_tol, C_t<R>* Rp, long sR, double* rn,
                                                       double* rnorm, const int* kact, int nlock,
                                                       double guard_tol) {
  const int j = blockIdx.x, k = blockIdx.y;
  if (kact && !kact[k]) return;  // converged k-point: its residuals stay as they were
  double2* S = Big + (long)k * sBig;
  const double2* kx = S + (mcols + j) * n3;      // KS block, column j (X part)
  const double2* ox = S + (2 * mcols + j) * n3;  // OS block, column j
  const double th = theta[k * s + j];
  C_t<R>* r = Rp + (long)k * sR + (long)j * n3;
  double a = 0, b = 0;
  for (long i = threadIdx.x; i < n3; i += 256) {
    const double2 o = ox[i];
    const double2 v = csub(kx[i], cscale(o, th));
    r[i] = mk<R>((R)v.x, (R)v.y);
    a += cabs2(v);
    b += cabs2(o);
  }
  __shared__ double sa[256], sb[256];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  const double rel = sqrt(sa[0]) / ((fabs(th) + sigma[k]) * sqrt(sb[0]) + 1e-300);
  if (threadIdx.x == 0) {
    rn[k * s + j] = rel;
    rnorm[k * s + j] = sqrt(sa[0]);
  }
  if (rel < (j < nlock ? act_tol : guard_tol)) {
    // Converged column: it stops feeding the search space (soft locking).  Its
    // preconditioned residual and its previous-direction column are zeroed, so the
    // next orthonormalisation drops them instead of amplifying rounding noise, and so
    // are the images of its search direction (K W, Omega W), which the operator
    // products then skip: the direction itself is zero.
    double2* pc = S + (2L * s + j) * n3;
    double2* wc = S + ((long)s + j) * n3;
    for (long i = threadIdx.x; i < n3; i += 256) {
      r[i] = mk<R>(0, 0);
      pc[i] = make_double2(0, 0);
      pc[mcols * n3 + i] = make_double2(0, 0);
      pc[2 * mcols * n3 + i] = make_double2(0, 0);
      wc[mcols * n3 + i] = make_double2(0, 0);
      wc[2 * mcols * n3 + i] = make_double2(0, 0);
    }
  }
}

template <typename R>
__global__ void widen_kernel(const C_t<R>* Rp, long sR, long n, double2* W, long sW, const int* kact) {
  const int k = blockIdx.y;
  if (kact && !kact[k]) return;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const C_t<R> v = Rp[(long)k * sR + e];
    W[(long)k * sW + e] = make_double2((double)v.x, (double)v.y);
  }
}

// Block-Jacobi preconditioner: W = D(k)^{-1} R with D(k) the 3 x 3 diagonal blocks of the
// pencil K(k) + sigma Omega, one per plane wave p (the p = q block of Eq. (4) in the sandwich
// form, from the diagonals of the k-shared operators and the wave vector K_p: never from
// K(k) itself).  Padding waves (p >= N) are identity.  R: n3 x s per k (k-stride sR,
// precision R); W: n3 x s per k in FP64 (ld n3, k-stride sW).  One thread per (wave, k).
// pairN = N > 0: R and W are in the paired basis (to_pair); the thread of a pair (p < c)
// takes both waves, D(k) being block diagonal in plane waves, not in the pairs.
// The inverse of wave p's block (symmetric positive definite) by its adjugate.
__device__ __forceinline__ void jacobi_block(double dm, double bm, double os, const double* kp, double c2,
                                             double sigma, double (&inv)[3][3]) {
  const double kk = kp[0] * kp[0] + kp[1] * kp[1] + kp[2] * kp[2];
  double a[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      a[i][j] = c2 * kp[i] * kp[j] * (dm / 3.0 + 0.5 * bm) + (i == j ? 0.5 * c2 * kk * bm + sigma * os : 0.0);
  inv[0][0] = a[1][1] * a[2][2] - a[1][2] * a[2][1];
  inv[0][1] = a[0][2] * a[2][1] - a[0][1] * a[2][2];
  inv[0][2] = a[0][1] * a[1][2] - a[0][2] * a[1][1];
  inv[1][0] = a[1][2] * a[2][0] - a[1][0] * a[2][2];
  inv[1][1] = a[0][0] * a[2][2] - a[0][2] * a[2][0];
  inv[1][2] = a[0][2] * a[1][0] - a[0][0] * a[1][2];
  inv[2][0] = a[1][0] * a[2][1] - a[1][1] * a[2][0];
  inv[2][1] = a[0][1] * a[2][0] - a[0][0] * a[2][1];
  inv[2][2] = a[0][0] * a[1][1] - a[0][1] * a[1][0];
  const double id = 1.0 / (a[0][0] * inv[0][0] + a[0][1] * inv[1][0] + a[0][2] * inv[2][0]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) inv[i][j] *= id;
}

__device__ __forceinline__ void apply3(const double (&inv)[3][3], const double2 (&v)[3], double2 (&o)[3]) {
  for (int i = 0; i < 3; ++i) {
    o[i] = make_double2(0, 0);
    for (int c = 0; c < 3; ++c) {
      o[i].x += inv[i][c] * v[c].x;
      o[i].y += inv[i][c] * v[c].y;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void jacobi_kernel(const double2* Dm, const double2* Bm, const double2* Os,
                                                      const double* Kv, int N, int Np, double c2,
                                                      const double* sigma, const C_t<R>* Rp, long sR, int s,
                                                      double2* W, long sW, const int* kact, int pairN) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (p >= Np || (kact && !kact[k])) return;
  const int cp = (pairN - 1) / 2;
  if (pairN > 0 && p > cp && p < pairN) return;  // the partner thread writes this row
  const long n3 = 3L * Np;
  const C_t<R>* r = Rp + (long)k * sR;
  double2* w = W + (long)k * sW;
  if (p >= N) {
    for (int j = 0; j < s; ++j)
      for (int c = 0; c < 3; ++c) {
        const C_t<R> v = r[j * n3 + c * Np + p];
        w[j * n3 + c * Np + p] = make_double2((double)v.x, (double)v.y);
      }
    return;
  }
  // the diagonal entries of Hermitian operators are real
  auto block = [&](int q, double (&inv)[3][3]) {
    jacobi_block(Dm[q + (long)q * Np].x, Bm[q + (long)q * Np].x, Os[q + (long)q * Np].x,
                 Kv + ((long)k * Np + q) * 3, c2, sigma[k], inv);
  };
  auto load = [&](int j, int q, double2 (&v)[3]) {
    for (int c = 0; c < 3; ++c) {
      const C_t<R> x = r[j * n3 + c * Np + q];
      v[c] = make_double2((double)x.x, (double)x.y);
    }
  };
  double inv[3][3];
  block(p, inv);
  if (pairN == 0 || p == cp) {
    for (int j = 0; j < s; ++j) {
      double2 v[3], o[3];
      load(j, p, v);
      apply3(inv, v, o);
      for (int c = 0; c < 3; ++c) w[j * n3 + c * Np + p] = o[c];
    }
    return;
  }
  const int pb = pairN - 1 - p;
  double invb[3][3];
  block(pb, invb);
  for (int j = 0; j < s; ++j) {
    double2 va[3], vb[3], oa[3], ob[3];
    load(j, p, va);
    load(j, pb, vb);
    for (int c = 0; c < 3; ++c) from_pair(va[c], vb[c]);
    apply3(inv, va, oa);
    apply3(invb, vb, ob);
    for (int c = 0; c < 3; ++c) {
      to_pair(oa[c], ob[c]);
      w[j * n3 + c * Np + p] = oa[c];
      w[j * n3 + c * Np + pb] = ob[c];
    }
  }
}

// Change of basis of vector blocks in place: dir > 0 plane waves -> paired basis (to_pair),
// dir < 0 back (from_pair).  X: n3 = 3 Np rows (three components of Np waves, the first N
// paired) x ncol per k (ld ldx, k-stride sX); T = float2 or double2, arithmetic in FP64.
template <typename T>
__global__ void pair_kernel(T* X, long ldx, long sX, int ncol, int N, int Np, int dir, const int* kact) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  const int c = (N - 1) / 2;
  if (p >= c || j >= ncol || (kact && !kact[k])) return;
  T* x = X + (long)k * sX + (long)j * ldx;
  const int pb = N - 1 - p;
  for (int d = 0; d < 3; ++d) {
    const T u = x[d * Np + p], v = x[d * Np + pb];
    double2 a = make_double2((double)u.x, (double)u.y), b = make_double2((double)v.x, (double)v.y);
    if (dir > 0) to_pair(a, b);
    else from_pair(a, b);
    x[d * Np + p].x = a.x;
    x[d * Np + p].y = a.y;
    x[d * Np + pb].x = b.x;
    x[d * Np + pb].y = b.y;
  }
}

// ---------------------------------------------------------------------------
// Omega_s X as a convolution.  Omega_s[p][q] = ghat_rho(n_p - n_q) (Eqs. (6)-(7); gather_kernel), so
// Omega_s x is the linear convolution of the density's Fourier table over the
// differences [-2M, 2M]^3 with the coefficients of x over [-M, M]^3; on the
// cyclic grid of L2 = 4M + 1 points per axis no difference wraps, so DFTs of
// length L2 along n3 and n2, a Toeplitz product along n1 (the table transformed
// along n2 and n3, Ch), and the inverse DFTs reproduce it exactly (up to
// rounding): about 0.7 MFLOP per column at M = 5 against 4 N^2 = 7 MFLOP for
// the dense real operator.
// ---------------------------------------------------------------------------

// Ch[d1][g2][g3] = L2^-2 sum_{d2, d3} T0[d1][d2][d3] exp(-i 2 pi (g2 (d2 - 2M) + g3 (d3 - 2M)) / L2):
// the density table T0 (first of the three tables of launch_dft) transformed along
// its last two axes, with the two inverse transforms' normalisation.
__global__ void omega_table_kernel(const double2* T0, int M, double2* Ch) {
  const int L2 = 4 * M + 1, M2 = 2 * M;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= L2 * L2 * L2) return;
  const int g3 = id % L2, g2 = (id / L2) % L2, d1 = id / (L2 * L2);
  double2 acc = make_double2(0, 0);
  for (int d2 = 0; d2 < L2; ++d2)
    for (int d3 = 0; d3 < L2; ++d3) {
      int j = (g2 * (d2 - M2) + g3 * (d3 - M2)) % L2;
      if (j < 0) j += L2;
      double s, c;
      sincospi(2.0 * j / L2, &s, &c);
      const double2 t = T0[((long)d1 * L2 + d2) * L2 + d3];
      acc.x += t.x * c + t.y * s;  // t exp(-i phi)
      acc.y += t.y * c - t.x * s;
    }
  Ch[id] = cscale(acc, 1.0 / ((double)L2 * L2));
}

struct ConvArgs {
  ConvCols c;
  const double2* Ch;
  int Np;
  double cs[21], sn[21];  // cos and sin of 2 pi j / L2, j < L2 (L2 <= 21)
};

// Length-L2 DFT, exp(-i 2 pi g m / L2), of L = 2M+1 coefficients at m = -M..M
// (x[M + m]) to out[g os], g < L2.  The pairs m, -m and g, L2 - g share their
// cosines and sines: X[g] = P - iQ and X[L2 - g] = P + iQ with
// P = x_0 + sum_m (x_m + x_-m) cos, Q = sum_m (x_m - x_-m) sin.
template <int M>
__device__ __forceinline__ void conv_fwd(const double2 (&x)[2 * M + 1], const ConvArgs& a, double2* out, int os) {
  constexpr int L2 = 4 * M + 1, H = 2 * M;
  double2 s[M], d[M];
  double2 f0 = x[M];
#pragma unroll
  for (int m = 1; m <= M; ++m) {
    s[m - 1] = cadd(x[M + m], x[M - m]);
    d[m - 1] = csub(x[M + m], x[M - m]);
    f0 = cadd(f0, s[m - 1]);
  }
  out[0] = f0;
#pragma unroll
  for (int g = 1; g <= H; ++g) {
    double2 P = x[M], Q = make_double2(0, 0);
#pragma unroll
    for (int m = 1; m <= M; ++m) {
      const double cv = a.cs[(g * m) % L2], sv = a.sn[(g * m) % L2];
      P.x = fma(s[m - 1].x, cv, P.x);
      P.y = fma(s[m - 1].y, cv, P.y);
      Q.x = fma(d[m - 1].x, sv, Q.x);
      Q.y = fma(d[m - 1].y, sv, Q.y);
    }
    out[g * os] = make_double2(P.x + Q.y, P.y - Q.x);
    out[(L2 - g) * os] = make_double2(P.x - Q.y, P.y + Q.x);
  }
}

// Inverse of conv_fwd restricted to n = -M..M (unnormalised): y[n] = sum_g Y[g]
// exp(+i 2 pi g n / L2) to out[(M + n) os]; y[n] = P + iQ, y[-n] = P - iQ with
// P = Y_0 + sum_g (Y_g + Y_-g) cos, Q = sum_g (Y_g - Y_-g) sin.
template <int M>
__device__ __forceinline__ void conv_inv(const double2 (&Y)[4 * M + 1], const ConvArgs& a, double2* out, int os) {
  constexpr int L2 = 4 * M + 1, H = 2 * M;
  double2 S[H], D[H];
  double2 y0 = Y[0];
#pragma unroll
  for (int g = 1; g <= H; ++g) {
    S[g - 1] = cadd(Y[g], Y[L2 - g]);
    D[g - 1] = csub(Y[g], Y[L2 - g]);
    y0 = cadd(y0, S[g - 1]);
  }
  out[M * os] = y0;
#pragma unroll
  for (int n = 1; n <= M; ++n) {
    double2 P = Y[0], Q = make_double2(0, 0);
#pragma unroll
    for (int g = 1; g <= H; ++g) {
      const double cv = a.cs[(g * n) % L2], sv = a.sn[(g * n) % L2];
      P.x = fma(S[g - 1].x, cv, P.x);
      P.y = fma(S[g - 1].y, cv, P.y);
      Q.x = fma(D[g - 1].x, sv, Q.x);
      Q.y = fma(D[g - 1].y, sv, Q.y);
    }
    out[(M + n) * os] = make_double2(P.x - Q.y, P.y + Q.x);
    out[(M - n) * os] = make_double2(P.x + Q.y, P.y - Q.x);
  }
}

// One workgroup per column of one component (Np rows, paired basis): the column is
// taken to plane waves, transformed along n3 (lines (a1, a2)) and n2 (lines (a1, g3)),
// multiplied along n1 by the Toeplitz matrix of the table Ch per line (g2, g3), transformed
// back along n2 and n3 and returned to the paired basis.  Every stage of one column
// lives in one LDS buffer of L L2^2 complex values; a stage reads its lines into
// registers, waits, and overwrites the buffer.  Rows N .. Np-1 (padding) are copied
// (the dense operator is the identity there).
template <int M>
__global__ __launch_bounds__(256, 2) void omega_conv_kernel(ConvArgs a) {
  constexpr int L = 2 * M + 1, L2 = 4 * M + 1, N = L * L * L, c = (N - 1) / 2, P2 = L2 * L2;
  static_assert(L * L2 <= 256, "one line per thread in the n2 and n3 stages");
  __shared__ double2 buf[L * P2];
  const int tid = threadIdx.x;
  const long u = blockIdx.x;
  const int e = a.c.bidx[u / a.c.ncolk];
  const long off = (long)(e / a.c.kdiv) * a.c.sB + (long)((e % a.c.kdiv) * a.c.ncolk + (int)(u % a.c.ncolk)) * a.c.ldb;
  const double2* x = a.c.X + off;
  double2* y = a.c.Y + off;

  // every load of the column in flight together, and the table line of this thread's
  // first n1 line (consumed three stages later) fetched meanwhile
  constexpr int NPR = (c + 256) / 256;  // pairs (p, N-1-p), p <= c, per thread
  double2 va[NPR], vb[NPR], t0[L2];
#pragma unroll
  for (int r = 0; r < NPR; ++r) {
    const int p = tid + r * 256;
    if (p < c) {
      va[r] = x[p];
      vb[r] = x[N - 1 - p];
    } else if (p == c) {
      va[r] = x[c];
    }
  }
  if (tid < P2)
#pragma unroll
    for (int dd = 0; dd < L2; ++dd) t0[dd] = a.Ch[(long)dd * P2 + tid];
  for (int r = N + tid; r < a.Np; r += 256) y[r] = x[r];
#pragma unroll
  for (int r = 0; r < NPR; ++r) {
    const int p = tid + r * 256;
    if (p < c) {
      from_pair(va[r], vb[r]);
      buf[p] = va[r];
      buf[N - 1 - p] = vb[r];
    } else if (p == c) {
      buf[c] = va[r];
    }
  }
  __syncthreads();
  {  // along n3: [a1][a2][a3] -> [a1][a2][g3]
    double2 v[L];
    const bool act = tid < L * L;
    if (act)
#pragma unroll
      for (int i = 0; i < L; ++i) v[i] = buf[tid * L + i];
    __syncthreads();
    if (act) conv_fwd<M>(v, a, buf + tid * L2, 1);
    __syncthreads();
  }
  {  // along n2: [a1][a2][g3] -> [a1][g2][g3]
    double2 v[L];
    const bool act = tid < L * L2;
    const int a1 = tid / L2, g3 = tid % L2;
    if (act)
#pragma unroll
      for (int i = 0; i < L; ++i) v[i] = buf[(a1 * L + i) * L2 + g3];
    __syncthreads();
    if (act) conv_fwd<M>(v, a, buf + a1 * P2 + g3, L2);
    __syncthreads();
  }
  // along n1: w[i] = sum_j Ch[i - j + 2M][g2][g3] v[j], in place per line l = g2 L2 + g3
  // (the first line of each thread with the table line fetched at the start)
#pragma unroll
  for (int rnd = 0; rnd < (P2 + 255) / 256; ++rnd) {
    const int l = tid + 256 * rnd;
    if (l < P2) {
      double2 v[L], w[L], t[L2];
#pragma unroll
      for (int i = 0; i < L; ++i) {
        v[i] = buf[i * P2 + l];
        w[i] = make_double2(0, 0);
      }
#pragma unroll
      for (int dd = 0; dd < L2; ++dd) t[dd] = rnd == 0 ? t0[dd] : a.Ch[(long)dd * P2 + l];
#pragma unroll
      for (int dd = 0; dd < L2; ++dd) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
          const int j = i + 2 * M - dd;
          if (j >= 0 && j < L) {
            w[i].x = fma(t[dd].x, v[j].x, w[i].x);
            w[i].x = fma(-t[dd].y, v[j].y, w[i].x);
            w[i].y = fma(t[dd].x, v[j].y, w[i].y);
            w[i].y = fma(t[dd].y, v[j].x, w[i].y);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < L; ++i) buf[i * P2 + l] = w[i];
    }
  }
  __syncthreads();
  {  // back along n2: [a1][g2][g3] -> [a1][a2][g3]
    double2 v[L2];
    const bool act = tid < L * L2;
    const int a1 = tid / L2, g3 = tid % L2;
    if (act)
#pragma unroll
      for (int i = 0; i < L2; ++i) v[i] = buf[(a1 * L2 + i) * L2 + g3];
    __syncthreads();
    if (act) conv_inv<M>(v, a, buf + a1 * L * L2 + g3, L2);
    __syncthreads();
  }
  {  // back along n3: [a1][a2][g3] -> [a1][a2][a3]
    double2 v[L2];
    const bool act = tid < L * L;
    if (act)
#pragma unroll
      for (int i = 0; i < L2; ++i) v[i] = buf[tid * L2 + i];
    __syncthreads();
    if (act) conv_inv<M>(v, a, buf + tid * L, 1);
    __syncthreads();
  }
  for (int p = tid; p <= c; p += 256) {
    if (p == c) {
      y[c] = buf[c];
    } else {
      double2 va = buf[p], vb = buf[N - 1 - p];
      to_pair(va, vb);
      y[p] = va;
      y[N - 1 - p] = vb;
    }
  }
}

// ---------------------------------------------------------------------------
// a8: adjoint.  Coefficients of the displacement (3) and Mandel stress (6)
// fields of selected Ritz vectors, on the (2M+1)^3 wave grid:
// Fc[col][f][p], col = k * nsel + j.
// ---------------------------------------------------------------------------
__global__ void field_coef_kernel(const double2* X, long ldx, long sX, int nsel, const double2* Zy,
                                  const double2* Zt, int N, int Np, double2* Fc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (p >= N) return;
  const double2* x = X + (long)k * sX + (long)j * ldx + p;
  const double2* z = Zy + (long)k * Np * 6 * nsel + (long)(6 * j) * Np + p;
  const double2 t3 = cscale(Zt[(long)k * Np * nsel + (long)j * Np + p], 1.0 / 3.0);
  double2* o = Fc + ((long)k * nsel + j) * 9 * N + p;
  o[0] = x[0];
  o[N] = x[Np];
  o[2 * N] = x[2 * Np];
  o[3 * N] = cadd(z[0], t3);
  o[4 * N] = cadd(z[Np], t3);
  o[5 * N] = cadd(z[2 * Np], t3);
  o[6 * N] = z[3 * Np];
  o[7 * N] = z[4 * Np];
  o[8 * N] = z[5 * Np];
}

// The synthesis phases exp(-i 2 pi m (i + 1/2) / nv), m = -M..M, i = 0..nv-1, as a table in
// dynamic LDS, [m + M][i], when (2M+1) nv <= SYNTH_PH (the launchers size the LDS); else
// each phase is computed where it is used.
constexpr int SYNTH_PH = 4096;
extern __shared__ double2 synth_ph[];
struct Phases {
  bool tab;
  int M, nv;
  __device__ __forceinline__ double2 operator()(int mi, int i) const {  // mi = m + M
    return tab ? synth_ph[mi * nv + i] : voxel_phase(mi - M, i, nv, -1);
  }
};
__device__ __forceinline__ Phases phase_table(int M, int nv) {
  const int n = (2 * M + 1) * nv;
  const bool tab = n <= SYNTH_PH;
  if (tab) {
    for (int e = threadIdx.x; e < n; e += blockDim.x) synth_ph[e] = voxel_phase(e / nv - M, e % nv, nv, -1);
    __syncthreads();
  }
  return Phases{tab, M, nv};
}
static inline size_t synth_lds(int M, int nv) {
  const long n = (2L * M + 1) * nv;
  return n <= SYNTH_PH ? (size_t)n * sizeof(double2) : 0;
}

// Synthesis g_e = sum_p c_p exp(-i 2 pi n_p . s_e), first two axes:
// H1[fc][n1][n2][i3] then H2[fc][n1][i2][i3] (fc = field x column).
__global__ void synth_pass1(const double2* Fc, int M, int nv, long nfc, double2* H1) {
  const Phases ph = phase_table(M, nv);
  const int L = 2 * M + 1;
  const long total = nfc * L * L * nv;
  const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int i3 = (int)(id % nv);
  const long r = id / nv;  // fc, n1, n2
  const double2* src = Fc + r * L;
  double2 acc = make_double2(0, 0);
  for (int n3 = 0; n3 < L; ++n3) acc = cadd(acc, cmul(ph(n3, i3), src[n3]));
  H1[id] = acc;
}

__global__ void synth_pass2(const double2* H1, int M, int nv, long nfc, double2* H2) {
  const Phases ph = phase_table(M, nv);
  const int L = 2 * M + 1;
  const long total = nfc * L * nv * nv;
  const long id = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (id >= total) return;
  const int i3 = (int)(id % nv);
  const int i2 = (int)((id / nv) % nv);
  const long fn1 = id / ((long)nv * nv);  // fc, n1
  const double2* src = H1 + fn1 * L * nv + i3;
  double2 acc = make_double2(0, 0);
  for (int n2 = 0; n2 < L; ++n2) acc = cadd(acc, cmul(ph(n2, i2), src[(long)n2 * nv]));
  H2[id] = acc;
}

// Last axis fused with the field energies:
//   d lambda / d rho_e = -v w'_e [ lambda Drho |u_e|^2
//        + (2 pi V)^2 ( Dcvol |tr sigma_e|^2 / 3 + Dcdev (|sigma_e|^2 - |tr sigma_e|^2 / 3) ) ]
// and d omega / d rho_e = lscale * (d lambda / d rho_e) / (2 omega_SI) (0 at omega = 0).
__global__ void energy_kernel(const double2* H2, int M, int nv, int ncols, const double* rho, MaterialND mat,
                              double v, double c2, const double* lam_nd, double lscale, double* out) {
  const Phases ph = phase_table(M, nv);
  const int L = 2 * M + 1;
  const long nvox = (long)nv * nv * nv;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (e >= nvox) return;
  const int i1 = (int)(e / ((long)nv * nv));
  const long i23 = e % ((long)nv * nv);
  double2 f[9];
  for (int q = 0; q < 9; ++q) {
    const double2* src = H2 + ((long)col * 9 + q) * L * nv * nv + i23;
    double2 acc = make_double2(0, 0);
    for (int n1 = 0; n1 < L; ++n1) acc = cadd(acc, cmul(ph(n1, i1), src[(long)n1 * nv * nv]));
    f[q] = acc;
  }
  const double u2 = cabs2(f[0]) + cabs2(f[1]) + cabs2(f[2]);
  const double2 tr = cadd(cadd(f[3], f[4]), f[5]);
  double s2 = 0;
  for (int q = 3; q < 9; ++q) s2 += cabs2(f[q]);
  const double t2 = cabs2(tr) / 3.0;
  const double lam = lam_nd[col];
  const double r = rho[e];
  const double wp = (mat.p == 1.0) ? 1.0 : mat.p * pow(r, mat.p - 1.0);
  const double dlam = -v * wp * (lam * mat.ddens * u2 + c2 * (mat.dcvol * t2 + mat.dcdev * (s2 - t2)));
  const double om = sqrt(fmax(lam, 0.0) * lscale);
  out[(long)col * nvox + e] = (lam > 0 && om > 0) ? lscale * dlam / (2.0 * om) : 0.0;
}

// The same two passes with each input slab read once: every output of a pass is an L-term
// sum over one axis, and the naive forms above read each input once per output along that
// axis (nv times), which leaves them bound by cache bandwidth.
// synth_pass1, one block per (fc, n1): the L x L coefficients Fc[fc][n1][.][.] into LDS after
// the phase table, then the L x nv outputs H1[fc][n1][n2][i3] (dynamic LDS L nv + L^2 entries).
__global__ void synth_pass1_slab(const double2* Fc, int M, int nv, double2* H1) {
  const int L = 2 * M + 1;
  double2* slab = synth_ph + L * nv;
  const long fn1 = blockIdx.x;  // fc, n1
  const double2* src = Fc + fn1 * L * L;
  for (int e = threadIdx.x; e < L * L; e += blockDim.x) slab[e] = src[e];
  const Phases ph = phase_table(M, nv);  // fills the table and synchronises
  double2* dst = H1 + fn1 * (long)L * nv;
  for (int e = threadIdx.x; e < L * nv; e += blockDim.x) {
    const int n2 = e / nv, i3 = e % nv;
    double2 acc = make_double2(0, 0);
    for (int n3 = 0; n3 < L; ++n3) acc = cadd(acc, cmul(ph(n3, i3), slab[n2 * L + n3]));
    dst[e] = acc;
  }
}

// synth_pass2, one block per (fc, n1): the L x nv slab H1[fc][n1][.][.] into LDS after the
// phase table, then all nv x nv outputs H2[fc][n1][i2][i3] from it (L nv <= SYNTH_SLAB, dynamic
// LDS 2 L nv entries).
constexpr int SYNTH_SLAB = 2048;
__global__ void synth_pass2_slab(const double2* H1, int M, int nv, double2* H2) {
  const int L = 2 * M + 1;
  double2* slab = synth_ph + L * nv;
  const long fn1 = blockIdx.x;  // fc, n1
  const double2* src = H1 + fn1 * L * nv;
  for (int e = threadIdx.x; e < L * nv; e += blockDim.x) slab[e] = src[e];
  const Phases ph = phase_table(M, nv);  // fills the table and synchronises
  double2* dst = H2 + fn1 * (long)nv * nv;
  for (int e = threadIdx.x; e < nv * nv; e += blockDim.x) {
    const int i2 = e / nv, i3 = e % nv;
    double2 acc = make_double2(0, 0);
    for (int n2 = 0; n2 < L; ++n2) acc = cadd(acc, cmul(ph(n2, i2), slab[n2 * nv + i3]));
    dst[e] = acc;
  }
}

// energy_kernel with a 16 x 16 tile of (i1, i23) voxels per block (i23 = i2 nv + i3): the
// 9 x L x 16 slab of H2 for the tile's i23 into LDS, read once per 16 values of i1.
constexpr int ENERGY_T = 16;
__global__ __launch_bounds__(256) void energy_slab_kernel(const double2* H2, int M, int nv, int ncols,
                                                          const double* rho, MaterialND mat, double v, double c2,
                                                          const double* lam_nd, double lscale, double* out) {
  double2* const synth_dyn = synth_ph;  // dynamic LDS: the phase table, then the slab
  const int L = 2 * M + 1;
  const long nvv = (long)nv * nv, nvox = nvv * nv;
  double2* slab = synth_dyn + L * nv;  // [q][n1][j], j < ENERGY_T
  for (int e = threadIdx.x; e < L * nv; e += blockDim.x) synth_dyn[e] = voxel_phase(e / nv - M, e % nv, nv, -1);
  const int col = blockIdx.y;
  const long t23 = blockIdx.x;                          // i23 tile
  const int ti1 = blockIdx.z;                           // i1 tile
  const long i23_0 = t23 * ENERGY_T;
  const double2* src = H2 + (long)col * 9 * L * nvv;
  for (int e = threadIdx.x; e < 9 * L * ENERGY_T; e += blockDim.x) {
    const int j = e % ENERGY_T, qn = e / ENERGY_T;      // qn = q L + n1
    const long i23 = i23_0 + j;
    slab[e] = i23 < nvv ? src[(long)qn * nvv + i23] : make_double2(0, 0);
  }
  __syncthreads();
  const int j = threadIdx.x % ENERGY_T, i1 = ti1 * ENERGY_T + threadIdx.x / ENERGY_T;
  const long i23 = i23_0 + j;
  if (i1 >= nv || i23 >= nvv) return;
  double2 f[9];
  for (int q = 0; q < 9; ++q) {
    double2 acc = make_double2(0, 0);
    for (int n1 = 0; n1 < L; ++n1) acc = cadd(acc, cmul(synth_dyn[n1 * nv + i1], slab[(q * L + n1) * ENERGY_T + j]));
    f[q] = acc;
  }
  const long e = (long)i1 * nvv + i23;
  const double u2 = cabs2(f[0]) + cabs2(f[1]) + cabs2(f[2]);
  const double2 tr = cadd(cadd(f[3], f[4]), f[5]);
  double s2 = 0;
  for (int q = 3; q < 9; ++q) s2 += cabs2(f[q]);
  const double t2 = cabs2(tr) / 3.0;
  const double lam = lam_nd[col];
  const double r = rho[e];
  const double wp = (mat.p == 1.0) ? 1.0 : mat.p * pow(r, mat.p - 1.0);
  const double dlam = -v * wp * (lam * mat.ddens * u2 + c2 * (mat.dcvol * t2 + mat.dcdev * (s2 - t2)));
  const double om = sqrt(fmax(lam, 0.0) * lscale);
  out[(long)col * nvox + e] = (lam > 0 && om > 0) ? lscale * dlam / (2.0 * om) : 0.0;
}

// grad_e = sum_col weight[col] * sens[col][e], summed in column order.
__global__ void weighted_sum_kernel(const double* sens, const double* wgt, int ncols, long nvox, double* grad) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= nvox) return;
  double acc = grad[e];
  for (int c = 0; c < ncols; ++c) acc += wgt[c] * sens[(long)c * nvox + e];
  grad[e] = acc;
}

// out[row][e] = sum_t coef[row][t] in[k next + t][e] with k = row / nsel: each requested
// (k, band) entry as a fixed combination of the computed columns of its k-point (the mean
// over a degenerate cluster); terms in column order, zero coefficients skipped.
__global__ void combine_cols_kernel(const double* in, int next, const double* coef, int nsel, long nvox, double* out) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= nvox) return;
  const int row = blockIdx.y, k = row / nsel;
  double acc = 0;
  for (int t = 0; t < next; ++t) {
    const double c = coef[(long)row * next + t];
    if (c != 0) acc += c * in[((long)k * next + t) * nvox + e];
  }
  out[(long)row * nvox + e] = acc;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_fields(const double* rho, int nvox, const MaterialND& mat, double* F, hipStream_t st) {
  hipLaunchKernelGGL(fields_kernel, dim3(nblk(nvox, 256)), dim3(256), 0, st, rho, nvox, mat, F);
}

void launch_dft(const double* F, int nv, int M, double v, double2* G1, double2* G2, double2* T, hipStream_t st) {
  const int M2 = 2 * M, L = 2 * M2 + 1, nf = 3;
  long n1 = (long)nf * nv * nv * L;
  hipLaunchKernelGGL(dft_pass1, dim3(nblk(n1, 256)), dim3(256), 0, st, F, nv, M2, G1, nf);
  long n2 = (long)nf * nv * L * L;
  hipLaunchKernelGGL(dft_pass2, dim3(nblk(n2, 256)), dim3(256), 0, st, G1, nv, M2, G2, nf);
  long n3 = (long)nf * L * L * L;
  hipLaunchKernelGGL(dft_pass3, dim3(nblk(n3, 256)), dim3(256), 0, st, G2, nv, M2, v, T, nf);
}

void launch_gather(const double2* T, int M, int N, int Np, double2* out, hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel, dim3(nblk(Np, 256), Np, 3), dim3(256), 0, st, T, M, N, Np, out);
}

void launch_split_inverse(double2* inv_v, double2* inv_d, long n, hipStream_t st) {
  hipLaunchKernelGGL(split_inverse_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, inv_v, inv_d, n);
}

void launch_identity(double2* X, int n, int batch, hipStream_t st) {
  hipLaunchKernelGGL(identity_kernel, dim3(nblk((long)n * n * batch, 256)), dim3(256), 0, st, X, n, batch);
}

void launch_kvec(const double* Q, const Recip& T, int M, int N, int Np, int nk, double* Kv, hipStream_t st) {
  hipLaunchKernelGGL(kvec_kernel, dim3(nblk(Np, 256), nk), dim3(256), 0, st, Q, T, M, N, Np, nk, Kv);
}

template <typename R>
void launch_assemble(const double2* Dm, const double2* Bm, const double2* Os, const double* Kv, int N, int Np,
                     int nk, double c2, const double* sigma, C_t<R>* A, long sA, int full, hipStream_t st) {
  const long nt = 3L * Np / 64;
  const long tiles = full ? nt * nt : nt * (nt + 1) / 2;
  hipLaunchKernelGGL((assemble_kernel<R>), dim3((unsigned)tiles), dim3(256), 0, st, Dm, Bm, Os, Kv, N, Np, nk,
                     c2, sigma, A, sA, full);
}
template void launch_assemble<double>(const double2*, const double2*, const double2*, const double*, int, int, int,
                                      double, const double*, double2*, long, int, hipStream_t);
template void launch_assemble<float>(const double2*, const double2*, const double2*, const double*, int, int, int,
                                     double, const double*, float2*, long, int, hipStream_t);

void launch_strain(const double2* X, long ldx, long sX, const double* Kv, int Np, int ncol, int nk, double2* Y,
                   double2* tr, hipStream_t st, const int* kact, int pairN, const int* cmask) {
  const long rows = pairN > 0 ? (pairN - 1) / 2 + 1 + (Np - pairN) : Np;  // threads per column
  hipLaunchKernelGGL(strain_kernel, dim3(nblk(rows, 256), ncol, nk), dim3(256), 0, st, X, ldx, sX, Kv, Np, ncol, Y,
                     tr, kact, pairN, cmask);
}

void launch_force(const double2* Zy, const double2* Zt, const double* Kv, int Np, int ncol, int nk, double c2,
                  double2* KX, long ldk, long sK, hipStream_t st, const int* kact, int pairN, const int* cmask) {
  const long rows = (pairN - 1) / 2 + 1 + (Np - pairN);  // threads per column
  hipLaunchKernelGGL(force_kernel, dim3(nblk(rows, 256), ncol, nk), dim3(256), 0, st, Zy, Zt, Kv, Np, ncol, c2, KX,
                     ldk, sK, kact, pairN, cmask);
}

void launch_realify(const double2* Mc, int N, int Np, double* Mr, hipStream_t st, const double2* Mc2) {
  const long n = (long)Np * Np;
  hipLaunchKernelGGL(realify_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Mc, Mc2, N, Np, Mr);
}

void launch_omega_table(const double2* T0, int M, double2* Ch, hipStream_t st) {
  const int L2 = 4 * M + 1, n = L2 * L2 * L2;
  hipLaunchKernelGGL(omega_table_kernel, dim3(nblk(n, 128)), dim3(128), 0, st, T0, M, Ch);
}

void launch_omega_conv(const ConvCols& c, int M, int Np, const double2* Ch, hipStream_t st, hipEvent_t ev0,
                       hipEvent_t ev1) {
  const long units = (long)c.nb * c.ncolk;
  if (units <= 0) return;
  ConvArgs a{};
  a.c = c;
  a.Ch = Ch;
  a.Np = Np;
  const int L2 = 4 * M + 1;
  for (int j = 0; j <= L2 / 2; ++j) {  // exactly even cosines and odd sines
    const double t = 2.0 * M_PI * j / L2;
    a.cs[j] = std::cos(t);
    a.sn[j] = std::sin(t);
    if (j > 0) {
      a.cs[L2 - j] = a.cs[j];
      a.sn[L2 - j] = -a.sn[j];
    }
  }
  const dim3 grid((unsigned)units), blk(256);
  // with ev0 set the launch records ev0 / ev1 at the kernel's start and end
#define PHX_CONV_LAUNCH(Mv)                                                                   \
  do {                                                                                        \
    if (ev0) hipExtLaunchKernelGGL(omega_conv_kernel<Mv>, grid, blk, 0, st, ev0, ev1, 0, a); \
    else hipLaunchKernelGGL(omega_conv_kernel<Mv>, grid, blk, 0, st, a);                      \
  } while (0)
  switch (M) {
    case 1: PHX_CONV_LAUNCH(1); break;
    case 2: PHX_CONV_LAUNCH(2); break;
    case 3: PHX_CONV_LAUNCH(3); break;
    case 4: PHX_CONV_LAUNCH(4); break;
    case 5: PHX_CONV_LAUNCH(5); break;
    default: break;
  }
#undef PHX_CONV_LAUNCH
}

void launch_zero(double2* X, long n, hipStream_t st) {
  unsigned nb = (unsigned)std::min<long>(nblk(n, 256), 8192);
  if (n > 0) hipLaunchKernelGGL(zero_kernel, dim3(nb), dim3(256), 0, st, X, n);
}

void launch_unit_columns(double2* X, long ldx, long sX, const int* idx, int s, int nk, hipStream_t st, int Np,
                         int pairN) {
  hipLaunchKernelGGL(unit_columns_kernel, dim3(nk), dim3(64), 0, st, X, ldx, sX, idx, s, Np, pairN);
}

template <typename T>
void launch_pair(T* X, long ldx, long sX, int ncol, int N, int Np, int nk, int dir, hipStream_t st, const int* kact) {
  const int c = (N - 1) / 2;
  if (c > 0 && ncol > 0 && nk > 0)
    hipLaunchKernelGGL((pair_kernel<T>), dim3(nblk(c, 256), ncol, nk), dim3(256), 0, st, X, ldx, sX, ncol, N, Np, dir,
                       kact);
}
template void launch_pair<double2>(double2*, long, long, int, int, int, int, int, hipStream_t, const int*);
template void launch_pair<float2>(float2*, long, long, int, int, int, int, int, hipStream_t, const int*);

template <typename R>
void launch_residual(double2* Big, long n3, long mcols, long sBig, const double* theta, int s, int nk,
                     const double* sigma, double act_tol, C_t<R>* Rp, long sR, double* rn, double* rnorm,
                     hipStream_t st, const int* kact, int nlock, double guard_tol) {
  if (nlock < 0 || nlock > s) nlock = s;
  hipLaunchKernelGGL((residual_kernel<R>), dim3(s, nk), dim3(256), 0, st, Big, n3, mcols, sBig, theta, s, sigma,
                     act_tol, Rp, sR, rn, rnorm, kact, nlock, guard_tol);
}
template void launch_residual<double>(double2*, long, long, long, const double*, int, int, const double*, double,
                                      double2*, long, double*, double*, hipStream_t, const int*, int, double);
template void launch_residual<float>(double2*, long, long, long, const double*, int, int, const double*, double,
                                     float2*, long, double*, double*, hipStream_t, const int*, int, double);

template <typename R>
void launch_widen(const C_t<R>* Rp, long sR, long n, double2* W, long sW, int nk, hipStream_t st, const int* kact) {
  unsigned nb = (unsigned)std::min<long>(nblk(n, 256), 4096);
  hipLaunchKernelGGL((widen_kernel<R>), dim3(nb, nk), dim3(256), 0, st, Rp, sR, n, W, sW, kact);
}
template void launch_widen<double>(const double2*, long, long, double2*, long, int, hipStream_t, const int*);

template <typename R>
void launch_jacobi(const double2* Dm, const double2* Bm, const double2* Os, const double* Kv, int N, int Np,
                   double c2, const double* sigma, const C_t<R>* Rp, long sR, int s, double2* W, long sW, int nk,
                   hipStream_t st, const int* kact, int pairN) {
  hipLaunchKernelGGL((jacobi_kernel<R>), dim3(nblk(Np, 256), nk), dim3(256), 0, st, Dm, Bm, Os, Kv, N, Np, c2, sigma,
                     Rp, sR, s, W, sW, kact, pairN);
}
template void launch_jacobi<double>(const double2*, const double2*, const double2*, const double*, int, int, double,
                                    const double*, const double2*, long, int, double2*, long, int, hipStream_t,
                                    const int*, int);
template void launch_jacobi<float>(const double2*, const double2*, const double2*, const double*, int, int, double,
                                   const double*, const float2*, long, int, double2*, long, int, hipStream_t,
                                   const int*, int);
template void launch_widen<float>(const float2*, long, long, double2*, long, int, hipStream_t, const int*);

void launch_field_coef(const double2* X, long ldx, long sX, int nsel, const double2* Zy, const double2* Zt, int N,
                       int Np, int nk, double2* Fc, hipStream_t st) {
  hipLaunchKernelGGL(field_coef_kernel, dim3(nblk(N, 256), nsel, nk), dim3(256), 0, st, X, ldx, sX, nsel, Zy, Zt,
                     N, Np, Fc);
}

// Coarse-to-fine embedding of displacement coefficient blocks: the plane wave n of
// order Mc keeps its coefficients at the same n in the order-M set (M > Mc); every
// other fine coefficient is zero (the destination is zeroed first).
__global__ void prolong_kernel(const double2* Xc, long ldc, long sXc, int Mc, int Npc, double2* X, long ldx, long sX,
                               int M, int Np) {
  const int Lc = 2 * Mc + 1, L = 2 * M + 1, Nc = Lc * Lc * Lc;
  const int pc = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y, k = blockIdx.z;
  if (pc >= Nc) return;
  const int n1 = pc / (Lc * Lc) - Mc, n2 = (pc / Lc) % Lc - Mc, n3 = pc % Lc - Mc;
  const int p = ((n1 + M) * L + (n2 + M)) * L + (n3 + M);
  const double2* src = Xc + (long)k * sXc + (long)j * ldc + pc;
  double2* dst = X + (long)k * sX + (long)j * ldx + p;
  for (int c = 0; c < 3; ++c) dst[(long)c * Np] = src[(long)c * Npc];
}

void launch_prolong(const double2* Xc, long ldc, long sXc, int Mc, int Npc, double2* X, long ldx, long sX, int M,
                    int Np, int s, int nk, hipStream_t st) {
  const int Lc = 2 * Mc + 1, Nc = Lc * Lc * Lc;
  hipLaunchKernelGGL(prolong_kernel, dim3(nblk(Nc, 256), s, nk), dim3(256), 0, st, Xc, ldc, sXc, Mc, Npc, X, ldx,
                     sX, M, Np);
}

// Xsel[k][:, j] = X[k][:, sel[j]] for n-row columns.
__global__ void gather_cols_kernel(const double2* X, long ldx, long sX, const int* sel, int nsel, long n,
                                   double2* Y, long sY) {
  const int j = blockIdx.y, k = blockIdx.z;
  const double2* src = X + (long)k * sX + (long)sel[j] * ldx;
  double2* dst = Y + (long)k * sY + (long)j * n;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) dst[i] = src[i];
}

void launch_gather_cols(const double2* X, long ldx, long sX, const int* sel, int nsel, long n, int nk, double2* Y,
                        long sY, hipStream_t st) {
  unsigned nb = (unsigned)std::min<long>(nblk(n, 256), 64);
  hipLaunchKernelGGL(gather_cols_kernel, dim3(nb, nsel, nk), dim3(256), 0, st, X, ldx, sX, sel, nsel, n, Y, sY);
}

void launch_synth(const double2* Fc, int M, int nv, long ncols, double2* H1, double2* H2, hipStream_t st) {
  const int L = 2 * M + 1;
  const long nfc = ncols * 9;
  const size_t lds = synth_lds(M, nv);
  if (lds > 0)
    hipLaunchKernelGGL(synth_pass1_slab, dim3((unsigned)(nfc * L)), dim3(256), lds + (size_t)L * L * sizeof(double2),
                       st, Fc, M, nv, H1);
  else
    hipLaunchKernelGGL(synth_pass1, dim3(nblk(nfc * L * L * nv, 256)), dim3(256), lds, st, Fc, M, nv, nfc, H1);
  if (lds > 0 && (long)L * nv <= SYNTH_SLAB)
    hipLaunchKernelGGL(synth_pass2_slab, dim3((unsigned)(nfc * L)), dim3(256), 2 * lds, st, H1, M, nv, H2);
  else
    hipLaunchKernelGGL(synth_pass2, dim3(nblk(nfc * L * nv * nv, 256)), dim3(256), lds, st, H1, M, nv, nfc, H2);
}

void launch_energy(const double2* H2, int M, int nv, int ncols, const double* rho, const MaterialND& mat, double v,
                   double c2, const double* lam_nd, double lscale, double* out, hipStream_t st) {
  const long nvox = (long)nv * nv * nv;
  const int L = 2 * M + 1;
  const size_t slab = ((size_t)L * nv + 9 * L * ENERGY_T) * sizeof(double2);
  if (slab <= 64 * 1024) {
    const long nvv = (long)nv * nv;
    const dim3 grid((unsigned)((nvv + ENERGY_T - 1) / ENERGY_T), (unsigned)ncols, (unsigned)((nv + ENERGY_T - 1) / ENERGY_T));
    hipLaunchKernelGGL(energy_slab_kernel, grid, dim3(256), slab, st, H2, M, nv, ncols, rho, mat, v, c2, lam_nd,
                       lscale, out);
  } else {
    hipLaunchKernelGGL(energy_kernel, dim3(nblk(nvox, 256), ncols), dim3(256), synth_lds(M, nv), st, H2, M, nv, ncols,
                       rho, mat, v, c2, lam_nd, lscale, out);
  }
}

void launch_weighted_sum(const double* sens, const double* wgt, int ncols, long nvox, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(weighted_sum_kernel, dim3(nblk(nvox, 256)), dim3(256), 0, st, sens, wgt, ncols, nvox, grad);
}

void launch_combine_cols(const double* in, int next, const double* coef, int nsel, int nk, long nvox, double* out,
                         hipStream_t st) {
  hipLaunchKernelGGL(combine_cols_kernel, dim3(nblk(nvox, 256), (unsigned)(nk * nsel)), dim3(256), 0, st, in, next,
                     coef, nsel, nvox, out);
}

}  // namespace phx
