// Launchers for the method-specific kernels (physics.hip) and the per-k small
// dense kernels (small.hip).
#pragma once
#include "phx_common.h"

namespace phx {

// Non-dimensional two-phase material, affine in w = rho^p.
struct MaterialND {
  double p;
  double dens0, ddens;  // density / rho_ref
  double cvol0, dcvol;  // 1/(3K) * E_ref   (Mandel volumetric compliance)
  double cdev0, dcdev;  // 1/(2G) * E_ref   (Mandel deviatoric compliance)
};

// Rows are the reciprocal vectors b_j of the unit-edge primitive cell.
struct Recip {
  double t[3][3];
};

void launch_fields(const double* rho, int nvox, const MaterialND& mat, double* F, hipStream_t st);
void launch_dft(const double* F, int nv, int M, double v, double2* G1, double2* G2, double2* T, hipStream_t st);
void launch_gather(const double2* T, int M, int N, int Np, double2* out, hipStream_t st);
void launch_split_inverse(double2* inv_v, double2* inv_d, long n, hipStream_t st);
void launch_identity(double2* X, int n, int batch, hipStream_t st);
void launch_kvec(const double* Q, const Recip& T, int M, int N, int Np, int nk, double* Kv, hipStream_t st);
template <typename R>
void launch_assemble(const double2* Dm, const double2* Bm, const double2* Os, const double* Kv, int N, int Np,
                     int nk, double c2, const double* sigma, C_t<R>* A, long sA, int full, hipStream_t st);
// kact (optional, device): per-k mask; k-points with kact[k] == 0 are skipped.
// pairN = 0 (strain only): Mandel strain (Np x 6 ncol per k) and trace (Np x ncol per k).
// pairN = N > 0: the displacement columns, the strain channels, the stresses and the
// forces are all in the paired basis of launch_realify (each wave n_p with -n_p), and the
// strain is split into five deviatoric channels (Np x 5 ncol per k) and the volumetric one
// (Np x ncol per k); the force kernel takes only this form (pairN = N required).
// cmask (optional, device, per k * ncol + j): columns whose entry is 0 are skipped.
void launch_strain(const double2* X, long ldx, long sX, const double* Kv, int Np, int ncol, int nk, double2* Y,
                   double2* tr, hipStream_t st, const int* kact = nullptr, int pairN = 0, const int* cmask = nullptr);
void launch_force(const double2* Zy, const double2* Zt, const double* Kv, int Np, int ncol, int nk, double c2,
                  double2* KX, long ldk, long sK, hipStream_t st, const int* kact, int pairN,
                  const int* cmask = nullptr);
// Mr = Re(U^H Mc U), U the unitary pairing each wave n_p with -n_p (see realify_kernel):
// real symmetric for the Fourier matrix of a real field and for its inverse.
// Mc2 (optional): the same for Mc + Mc2.
void launch_realify(const double2* Mc, int N, int Np, double* Mr, hipStream_t st, const double2* Mc2 = nullptr);
void launch_zero(double2* X, long n, hipStream_t st);
// Omega_s times listed columns as an exact convolution with the density's Fourier
// table (orders M <= OMEGA_CONV_MAX_M; the same product as the dense real operator
// Re(U^H Omega_s U) in the paired basis, rows N .. Np-1 copied).  Column u < nb ncolk:
// e = bidx[u / ncolk], stored at (e / kdiv) sB + ((e % kdiv) ncolk + u % ncolk) ldb in X
// (input) and Y (output, not aliasing X), Np rows each.  Ch: launch_omega_table's
// (4M+1)^3 table of the design.
struct ConvCols {
  const double2* X;
  double2* Y;
  long sB, ldb;
  int nb, ncolk, kdiv;
  const int* bidx;
};
constexpr int OMEGA_CONV_MAX_M = 5;
// T0: the density table of launch_dft ((4M+1)^3, differences -2M..2M per axis).
void launch_omega_table(const double2* T0, int M, double2* Ch, hipStream_t st);
// ev0 / ev1 (optional): events the launch records at the kernel's start and end.
void launch_omega_conv(const ConvCols& c, int M, int Np, const double2* Ch, hipStream_t st, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// pairN = N > 0: the unit columns in the paired basis (launch_realify); Np: rows per component.
void launch_unit_columns(double2* X, long ldx, long sX, const int* idx, int s, int nk, hipStream_t st, int Np,
                         int pairN);
// Vector blocks (3 Np rows per column, ncol columns per k) to the paired basis in place
// (dir > 0) or back to plane waves (dir < 0); k-points with kact[k] == 0 are skipped.
template <typename T>
void launch_pair(T* X, long ldx, long sX, int ncol, int N, int Np, int nk, int dir, hipStream_t st,
                 const int* kact = nullptr);
void launch_prolong(const double2* Xc, long ldc, long sXc, int Mc, int Npc, double2* X, long ldx, long sX, int M,
                    int Np, int s, int nk, hipStream_t st);
// Columns j >= nlock (the guard vectors beyond the wanted bands) lock below guard_tol
// instead of act_tol (nlock = s: every column at act_tol).
template <typename R>
void launch_residual(double2* Big, long n3, long mcols, long sBig, const double* theta, int s, int nk,
                     const double* sigma, double act_tol, C_t<R>* Rp, long sR, double* rn, double* rnorm,
                     hipStream_t st, const int* kact = nullptr, int nlock = -1, double guard_tol = 0.0);
template <typename R>
void launch_widen(const C_t<R>* Rp, long sR, long n, double2* W, long sW, int nk, hipStream_t st,
                  const int* kact = nullptr);
// W = D(k)^{-1} R, D(k) the 3 x 3 per-wave diagonal blocks of K(k) + sigma Omega (block Jacobi).
template <typename R>
void launch_jacobi(const double2* Dm, const double2* Bm, const double2* Os, const double* Kv, int N, int Np,
                   double c2, const double* sigma, const C_t<R>* Rp, long sR, int s, double2* W, long sW, int nk,
                   hipStream_t st, const int* kact = nullptr, int pairN = 0);
void launch_field_coef(const double2* X, long ldx, long sX, int nsel, const double2* Zy, const double2* Zt, int N,
                       int Np, int nk, double2* Fc, hipStream_t st);
void launch_gather_cols(const double2* X, long ldx, long sX, const int* sel, int nsel, long n, int nk, double2* Y,
                        long sY, hipStream_t st);
void launch_synth(const double2* Fc, int M, int nv, long ncols, double2* H1, double2* H2, hipStream_t st);
void launch_energy(const double2* H2, int M, int nv, int ncols, const double* rho, const MaterialND& mat, double v,
                   double c2, const double* lam_nd, double lscale, double* out, hipStream_t st);
void launch_weighted_sum(const double* sens, const double* wgt, int ncols, long nvox, double* grad, hipStream_t st);
// out[(k nsel + j)][e] = sum_t coef[(k nsel + j) next + t] in[(k next + t)][e], for k < nk, j < nsel.
void launch_combine_cols(const double* in, int next, const double* coef, int nsel, int nk, long nvox, double* out,
                         hipStream_t st);

// design.hip: Heaviside projection of a (reduced, optionally octant-mirrored) design field.
void launch_project(int nv, int sp, double r, double beta, int oct, const double* x, double* rho, hipStream_t st);
void launch_project_adjoint(int nv, int sp, double r, double beta, int oct, const double* x, const double* grad_rho,
                            double* coef, double* grad_x, hipStream_t st);

// small.hip: per-k dense kernels on m x m (m <= 64) Gram matrices, FP64.
void launch_chol_drop(const double2* G, int m, int nk, double drop, double2* C0, int* keep, hipStream_t st,
                      const int* kact = nullptr);
// Cx, Cp: m x s per k at k-stride sCx (0: m s).  method 0: cyclic Jacobi on the projected
// matrix (eigenvalues to high relative accuracy); 1: Householder tridiagonalisation,
// multisection and inverse iteration (absolute accuracy eps ||A||; s <= 24, else Jacobi).
void launch_rr_gen(const double2* G2, int m, int s, int nk, double drop, double2* C0, int* keep, double2* Cx,
                   double2* Cp, double* theta, int* sweeps, hipStream_t st, const int* kact = nullptr,
                   long sCx = 0, int method = 0);
void launch_rr_eig(const double2* G, const int* keep, int m, int s, int nk, double2* C, double* theta,
                   int* sweeps, hipStream_t st, const int* kact = nullptr);

}  // namespace phx
