// Host-side logic of the phx library that touches no GPU: argument validation, the
// lattice geometry, the Brillouin-zone path, the k-chunk sizing, the grouping of k-points
// that share a preconditioner factor, and the plan that turns degenerate clusters of Ritz
// values into cluster-mean sensitivities.  Plain C++ (no HIP types) so that it also builds
// with the host compiler alone, under the address and undefined-behaviour sanitizers.
#pragma once

#include <vector>

#include "../../include/phx.h"

namespace phx_host {

// Primitive lattice vectors (rows, in units of the cube edge a) of SC, BCC and FCC.
void prim_rows(int lattice, double A[3][3]);

// Reciprocal rows T (a_i . t_j = delta_ij, no 2 pi) of the rows A; returns |det A|.
double reciprocal(const double A[3][3], double T[3][3]);

// Each check returns nullptr when the arguments are valid, else the reason.
const char* check_cell(const phx_cell* c);
const char* check_rho(const double* rho, long n);
const char* check_q(const double* q, int nk);
// block_opt: the option "block" (0 = automatic).
const char* check_bands(const phx_cell* c, int nb, int nsens, const int* band_no, int block_opt);
// The node layout of a design projection alone, and with its radius and Heaviside
// parameter; on success *ndesign (may be NULL) receives the number of design variables.
const char* projection_shape(const phx_projection* p, long* ndesign);
const char* check_projection(const phx_projection* p, long* ndesign);

// k-points along the named path through the irreducible Brillouin zone (reduced
// coordinates with respect to the reciprocal rows), as documented for phx_kpath.
int kpath(int lattice, const char* path, int nk, double* q_out);

// Search block s of the eigensolver for nb wanted bands of an order with N plane waves.
int choose_block(int block_opt, int nb, int N);

// Device bytes per k-point of a solve: the pencil factors (absent with the block-Jacobi
// preconditioner, precond 1), the basis [X W P] with its K and Omega images, the
// preconditioned block, and the per-plane-wave strain and stress channels.
long per_k_bytes(long n3, long Np, int s, int prec, int precond);

// k-points per chunk: as many as mem_gb holds at `per` bytes each, at least one.
int chunk_size(int nk, double mem_gb, long per);

// Groups of consecutive k-points (among those with which[k] != 0) that share one pencil
// factor: a k-point joins the group of the last leader l when k - l < kmax, |k - l| (the
// Cartesian distance of the wave vectors qcart, 3 per k) <= dist and <= rel times the
// shorter of |k| and |l|.  fmap[k] (for which[k] != 0) receives f0 + its group's index;
// the leaders are appended to lead.  Returns the number of groups.
int share_groups(const double* qcart, int nk, const char* which, int kmax, double dist, double rel, int f0,
                 int* fmap, std::vector<int>& lead);

// Degenerate-cluster plan of one chunk.  theta: nk x s Ritz values (ascending per k);
// sel: the nsel requested band indices (0-based, < s).  The cluster of band b at k is the
// run of neighbours whose frequencies sqrt(theta) differ by less than dtol relative;
// each requested (k, band) whose cluster has more than one member receives the mean
// derivative of the cluster.  ext lists the bands whose derivatives are needed (sel, or
// the union of sel and the clusters); coef (nk x nsel x ext.size()) holds the weights
// that turn those derivatives into the reported ones.  ndeg counts the requested
// entries that lie in a cluster (0: ext == sel and coef is empty).
struct ClusterPlan {
  long ndeg = 0;
  std::vector<int> lo, hi;  // cluster bounds, nk x nsel
  std::vector<int> ext;
  std::vector<double> coef;
};
ClusterPlan cluster_plan(const double* theta, int nk, int s, const int* sel, int nsel, double dtol);

}  // namespace phx_host
