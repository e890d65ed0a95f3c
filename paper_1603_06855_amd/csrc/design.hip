// Design-variable projection of the topology optimisation (section "Topology
// optimization formulation": the Heaviside projection method with a reduced design
// variable field, continuation on its sharpness, and the reflection symmetry the SC
// designs are optimised with, section "Study of cubic unit cells").
//
// Elements (voxels) e = (i1, i2, i3) of an nv^3 grid, centroids at (i + 1/2) in element
// widths along the primitive axes.  Design nodes every `sp` elements: node j sits at the
// centre of the sp^3 block of elements sp j .. sp j + sp - 1, i.e. at sp j + sp/2.  With
// the octant option the node values are given on nodes j < nn/2 per axis (nn = nv / sp)
// and mirrored, node j taking the value of node nn - 1 - j, which reflects the design
// about the cell's mid-planes.  Per element:
//   w_en = max(0, r - |x_e - x_n|)   (periodic minimum image, element widths)
//   mu_e = sum_n w_en d_n / sum_n w_en
//   rho_e = 1 - exp(-beta mu_e) + mu_e exp(-beta)
#include "phx_common.h"
#include "phx_physics.h"

namespace phx {

struct ProjGeom {
  int nv, sp, nn, oct;
  double r, beta;
};

__device__ __forceinline__ int wrapi(int j, int n) { return ((j % n) + n) % n; }

// index of full-grid node (j1, j2, j3) in the design array
__device__ __forceinline__ long design_index(const ProjGeom& g, int j1, int j2, int j3) {
  if (!g.oct) return ((long)j1 * g.nn + j2) * g.nn + j3;
  const int h = g.nn / 2;
  j1 = j1 < h ? j1 : g.nn - 1 - j1;
  j2 = j2 < h ? j2 : g.nn - 1 - j2;
  j3 = j3 < h ? j3 : g.nn - 1 - j3;
  return ((long)j1 * h + j2) * h + j3;
}

// Nodes whose centre lies within r of position c (element widths) along one axis: the
// unwrapped node indices lo .. hi.
__device__ __forceinline__ void node_range(const ProjGeom& g, double c, int& lo, int& hi) {
  lo = (int)ceil((c - g.r - 0.5 * g.sp) / g.sp);
  hi = (int)floor((c + g.r - 0.5 * g.sp) / g.sp);
}

// mu_e and W_e = sum_n w_en for element e.
__device__ void element_filter(const ProjGeom& g, const double* x, int i1, int i2, int i3, double& mu,
                               double& W) {
  const double c1 = i1 + 0.5, c2 = i2 + 0.5, c3 = i3 + 0.5;
  int a1, b1, a2, b2, a3, b3;
  node_range(g, c1, a1, b1);
  node_range(g, c2, a2, b2);
  node_range(g, c3, a3, b3);
  double s = 0, w = 0;
  for (int j1 = a1; j1 <= b1; ++j1) {
    const double d1 = c1 - (g.sp * j1 + 0.5 * g.sp);
    for (int j2 = a2; j2 <= b2; ++j2) {
      const double d2 = c2 - (g.sp * j2 + 0.5 * g.sp);
      for (int j3 = a3; j3 <= b3; ++j3) {
        const double d3 = c3 - (g.sp * j3 + 0.5 * g.sp);
        const double wt = g.r - sqrt(d1 * d1 + d2 * d2 + d3 * d3);
        if (wt > 0) {
          w += wt;
          s += wt * x[design_index(g, wrapi(j1, g.nn), wrapi(j2, g.nn), wrapi(j3, g.nn))];
        }
      }
    }
  }
  W = w;
  mu = s / w;
}

__global__ void project_kernel(ProjGeom g, const double* x, double* rho, double* coef, const double* grad) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long ne = (long)g.nv * g.nv * g.nv;
  if (e >= ne) return;
  const int i1 = (int)(e / ((long)g.nv * g.nv)), i2 = (int)((e / g.nv) % g.nv), i3 = (int)(e % g.nv);
  double mu, W;
  element_filter(g, x, i1, i2, i3, mu, W);
  const double eb = exp(-g.beta);
  if (rho) rho[e] = 1.0 - exp(-g.beta * mu) + mu * eb;
  // adjoint pass: c_e = (d rho_e / d mu_e) grad_e / W_e
  if (coef) coef[e] = (g.beta * exp(-g.beta * mu) + eb) * grad[e] / W;
}

// grad_x for one design variable: the sum over its node (and, with the octant, its seven
// mirror images) of sum_e w_en c_e.
__global__ void project_adjoint_kernel(ProjGeom g, const double* coef, double* gx) {
  const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const int nd = g.oct ? g.nn / 2 : g.nn;
  if (t >= (long)nd * nd * nd) return;
  const int k1 = (int)(t / ((long)nd * nd)), k2 = (int)((t / nd) % nd), k3 = (int)(t % nd);
  const int nim = g.oct ? 2 : 1;
  double acc = 0;
  for (int m1 = 0; m1 < nim; ++m1)
    for (int m2 = 0; m2 < nim; ++m2)
      for (int m3 = 0; m3 < nim; ++m3) {
        const int j1 = m1 ? g.nn - 1 - k1 : k1, j2 = m2 ? g.nn - 1 - k2 : k2, j3 = m3 ? g.nn - 1 - k3 : k3;
        const double p1 = g.sp * j1 + 0.5 * g.sp, p2 = g.sp * j2 + 0.5 * g.sp, p3 = g.sp * j3 + 0.5 * g.sp;
        // elements with centroid within r of the node: unwrapped indices
        const int a1 = (int)ceil(p1 - g.r - 0.5), b1 = (int)floor(p1 + g.r - 0.5);
        const int a2 = (int)ceil(p2 - g.r - 0.5), b2 = (int)floor(p2 + g.r - 0.5);
        const int a3 = (int)ceil(p3 - g.r - 0.5), b3 = (int)floor(p3 + g.r - 0.5);
        for (int i1 = a1; i1 <= b1; ++i1) {
          const double d1 = i1 + 0.5 - p1;
          for (int i2 = a2; i2 <= b2; ++i2) {
            const double d2 = i2 + 0.5 - p2;
            for (int i3 = a3; i3 <= b3; ++i3) {
              const double d3 = i3 + 0.5 - p3;
              const double wt = g.r - sqrt(d1 * d1 + d2 * d2 + d3 * d3);
              if (wt > 0)
                acc += wt * coef[((long)wrapi(i1, g.nv) * g.nv + wrapi(i2, g.nv)) * g.nv + wrapi(i3, g.nv)];
            }
          }
        }
      }
  gx[t] = acc;
}

static ProjGeom geom(int nv, int sp, double r, double beta, int oct) {
  ProjGeom g;
  g.nv = nv;
  g.sp = sp;
  g.nn = nv / sp;
  g.oct = oct;
  g.r = r;
  g.beta = beta;
  return g;
}

void launch_project(int nv, int sp, double r, double beta, int oct, const double* x, double* rho, hipStream_t st) {
  const ProjGeom g = geom(nv, sp, r, beta, oct);
  const long ne = (long)nv * nv * nv;
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, g, x, rho,
                     (double*)nullptr, (const double*)nullptr);
}

void launch_project_adjoint(int nv, int sp, double r, double beta, int oct, const double* x, const double* grad_rho,
                            double* coef, double* grad_x, hipStream_t st) {
  const ProjGeom g = geom(nv, sp, r, beta, oct);
  const long ne = (long)nv * nv * nv;
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, st, g, x, (double*)nullptr,
                     coef, grad_rho);
  const int nd = oct ? g.nn / 2 : g.nn;
  const long nx = (long)nd * nd * nd;
  hipLaunchKernelGGL(project_adjoint_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, g,
                     (const double*)coef, grad_x);
}

}  // namespace phx
