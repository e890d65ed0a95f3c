// Host-side logic of the phx library (no GPU calls): validation, lattice geometry, the
// Brillouin-zone path, chunk sizing, factor-sharing groups and degenerate-cluster plans,
// plus the C entry points that need nothing else (phx_validate, phx_kpath,
// phx_projection_size).
#include "phx_host.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <string>

static_assert(sizeof(phx_lattice) == sizeof(int), "the C enum phx_lattice is int-sized");

namespace phx_host {

void prim_rows(int lattice, double A[3][3]) {
  static const double sc[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  static const double bcc[3][3] = {{-0.5, 0.5, 0.5}, {0.5, -0.5, 0.5}, {0.5, 0.5, -0.5}};
  static const double fcc[3][3] = {{0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};
  const double(*s)[3] = lattice == PHX_SC ? sc : (lattice == PHX_BCC ? bcc : fcc);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = s[i][j];
}

double reciprocal(const double A[3][3], double T[3][3]) {
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                     A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  // inverse of A, then transpose: T[j][c] = inv(A)[c][j]
  double inv[3][3];
  inv[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
  inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
  inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
  inv[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
  inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
  inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
  inv[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
  inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
  inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) T[j][c] = inv[c][j];
  return fabs(det);
}

static bool material_ok(const phx_material& m) {
  return isfinite(m.density) && isfinite(m.youngs) && isfinite(m.poisson) && m.density > 0 && m.youngs > 0 &&
         m.poisson > -1.0 && m.poisson < 0.5;
}

const char* check_cell(const phx_cell* c) {
  if (!c) return "cell is NULL";
  // a C caller may store any int in the enum field; reading it as the enum type would be
  // undefined behaviour in C++ for values outside the enumerators' range
  int lattice;
  memcpy(&lattice, &c->lattice, sizeof lattice);
  if (lattice < PHX_SC || lattice > PHX_FCC) return "unknown lattice";
  if (!(c->a > 0) || !isfinite(c->a)) return "cube edge a must be positive";
  if (c->M < 1 || c->M > 8) return "plane-wave order M must be in [1, 8]";
  if (c->nv < 2 * c->M + 1) return "nv must be at least 2M+1 (the centroid rule aliases otherwise)";
  if (c->nv > 256) return "nv must be at most 256";
  if (!material_ok(c->phase0) || !material_ok(c->phase1))
    return "material needs density > 0, Young's modulus > 0, Poisson ratio in (-1, 1/2)";
  if (!(c->simp_p >= 1.0) || !isfinite(c->simp_p)) return "simp_p must be >= 1";
  return nullptr;
}

const char* check_rho(const double* rho, long n) {
  if (!rho) return "rho is NULL";
  for (long e = 0; e < n; ++e)
    if (!isfinite(rho[e]) || rho[e] < 0) return "rho must be finite and non-negative";
  return nullptr;
}

const char* check_q(const double* q, int nk) {
  if (nk < 1) return "nk must be positive";
  if (!q) return "q is NULL";
  for (long i = 0; i < 3L * nk; ++i)
    if (!isfinite(q[i])) return "q must be finite";
  return nullptr;
}

const char* check_bands(const phx_cell* c, int nb, int nsens, const int* band_no, int block_opt) {
  const long L = 2L * c->M + 1, n3 = 3 * L * L * L;
  if (nb < 1 || nb > 16 || nb > n3) return "nbands must be in [1, min(16, 3N)]";
  if (block_opt > 0 && block_opt <= nb && block_opt < n3)
    return "option block must exceed nbands (the search block holds the wanted bands and guards)";
  if (nsens < 0) return "nsens must be non-negative";
  if (nsens > 0 && !band_no) return "band_no is NULL";
  for (int j = 0; j < nsens; ++j)
    if (band_no[j] < 1 || band_no[j] > nb) return "band_no entries must be in [1, nbands]";
  return nullptr;
}

const char* projection_shape(const phx_projection* p, long* ndesign) {
  if (!p) return "projection is NULL";
  if (p->nv < 2 || (p->spacing != 1 && p->spacing != 2) || p->nv % p->spacing)
    return "nv must be a positive multiple of spacing (1 or 2)";
  const long nn = p->nv / p->spacing;
  if (p->octant && nn % 2) return "the octant needs an even number of design nodes per axis";
  const long nd = p->octant ? nn / 2 : nn;
  if (ndesign) *ndesign = nd * nd * nd;
  return nullptr;
}

const char* check_projection(const phx_projection* p, long* ndesign) {
  if (const char* e = projection_shape(p, ndesign)) return e;
  const double rmin = p->spacing == 2 ? 0.8660254037844387 : 0.0;  // farthest element centroid from a node
  if (!(p->radius > rmin) || !(2.0 * p->radius + p->spacing < p->nv))
    return "radius must reach the nearest design node and stay below half the cell";
  if (!(p->beta >= 0) || !(p->beta <= 1e3)) return "beta must lie in [0, 1000]";
  return nullptr;
}

int kpath(int lattice, const char* path, int nk, double* q_out) {
  if (!q_out || lattice < PHX_SC || lattice > PHX_FCC) return PHX_EINVAL;
  // high-symmetry points in conventional-cube units (cycles per a)
  struct Pt {
    char c;
    double x, y, z;
  };
  static const Pt sc[] = {{'G', 0, 0, 0}, {'X', 0, 0.5, 0}, {'M', 0.5, 0.5, 0}, {'R', 0.5, 0.5, 0.5}};
  static const Pt bcc[] = {{'G', 0, 0, 0}, {'H', 0, 0, 1}, {'N', 0.5, 0.5, 0}, {'P', 0.5, 0.5, 0.5}};
  static const Pt fcc[] = {{'G', 0, 0, 0},       {'X', 0, 1, 0},         {'W', 0.5, 1, 0},
                           {'K', 0.75, 0.75, 0}, {'L', 0.5, 0.5, 0.5}, {'U', 0.25, 1, 0.25}};
  const Pt* tab = lattice == PHX_SC ? sc : (lattice == PHX_BCC ? bcc : fcc);
  const int ntab = lattice == PHX_FCC ? 6 : 4;
  const char* def = lattice == PHX_SC ? "GXMGRX|MR" : (lattice == PHX_BCC ? "GHNGPH|PN" : "GXWKGLUWLK|UX");
  const std::string p = path ? path : def;
  // branches of vertices ('|' starts a new branch)
  std::vector<std::vector<const Pt*>> br(1);
  for (char ch : p) {
    if (ch == '|') {
      br.emplace_back();
      continue;
    }
    const Pt* f = nullptr;
    for (int i = 0; i < ntab; ++i)
      if (tab[i].c == ch) f = &tab[i];
    if (!f) return PHX_EINVAL;
    br.back().push_back(f);
  }
  br.erase(std::remove_if(br.begin(), br.end(), [](const std::vector<const Pt*>& b) { return b.empty(); }),
           br.end());
  int nvert = 0;
  for (auto& b : br) nvert += (int)b.size();
  if (nvert == 0 || nk < nvert) return PHX_EINVAL;
  std::vector<double> len;
  for (auto& b : br)
    for (size_t i = 0; i + 1 < b.size(); ++i) {
      const double dx = b[i + 1]->x - b[i]->x, dy = b[i + 1]->y - b[i]->y, dz = b[i + 1]->z - b[i]->z;
      len.push_back(sqrt(dx * dx + dy * dy + dz * dz));
    }
  // the points beyond the vertices go to the segments in proportion to their lengths,
  // the remainder of the rounding to the largest fractional shares
  const int extra = nk - nvert;
  std::vector<int> cnt(len.size(), 0);
  const double tot = std::accumulate(len.begin(), len.end(), 0.0);
  if (!len.empty() && tot > 0) {
    std::vector<double> share(len.size());
    int used = 0;
    for (size_t i = 0; i < len.size(); ++i) {
      share[i] = extra * len[i] / tot;
      cnt[i] = (int)floor(share[i]);
      used += cnt[i];
    }
    std::vector<size_t> ord(len.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](size_t a, size_t b) { return (share[a] - cnt[a]) > (share[b] - cnt[b]); });
    for (int r = 0; r < extra - used; ++r) cnt[ord[r]]++;
  } else if (extra > 0) {
    return PHX_EINVAL;
  }
  // cube units -> reduced coordinates: q_j = a_j . k
  double A[3][3];
  prim_rows(lattice, A);
  int o = 0;
  size_t si = 0;
  auto emit = [&](double x, double y, double z) {
    for (int j = 0; j < 3; ++j) q_out[3 * o + j] = A[j][0] * x + A[j][1] * y + A[j][2] * z;
    ++o;
  };
  for (auto& b : br) {
    emit(b[0]->x, b[0]->y, b[0]->z);
    for (size_t i = 0; i + 1 < b.size(); ++i, ++si) {
      const Pt *u = b[i], *v = b[i + 1];
      const int c = cnt[si];
      for (int j = 1; j <= c; ++j) {
        const double t = (double)j / (c + 1);
        emit(u->x + (v->x - u->x) * t, u->y + (v->y - u->y) * t, u->z + (v->z - u->z) * t);
      }
      emit(v->x, v->y, v->z);
    }
  }
  return o == nk ? PHX_OK : PHX_EINVAL;
}

int choose_block(int block_opt, int nb, int N) {
  const int s = block_opt > 0 ? block_opt : std::min(21, nb + std::max(8, nb));
  return std::min(s, 3 * N);
}

long per_k_bytes(long n3, long Np, int s, int prec, int precond) {
  const long m = 3L * s;
  const long pc = prec == PHX_FP64 ? 16 : 8;
  const long ws = prec == PHX_FP64 ? 128 : 256;
  const long factor = precond == 1 ? 0 : n3 * n3 * pc + (n3 / 64) * 4096 * pc + ((n3 + ws - 1) / ws) * ws * ws * pc;
  return factor + 3L * n3 * m * 16 + 2L * n3 * s * pc + 4L * Np * 7 * s * 16;
}

int chunk_size(int nk, double mem_gb, long per) {
  const double fit = mem_gb * 1073741824.0 / (double)std::max(per, 1L);
  return (int)std::max(1.0, std::min((double)nk, floor(fit)));
}

int share_groups(const double* qcart, int nk, const char* which, int kmax, double dist, double rel, int f0,
                 int* fmap, std::vector<int>& lead) {
  const size_t first = lead.size();
  for (int k = 0; k < nk; ++k) {
    if (!which[k]) continue;
    bool join = false;
    if (lead.size() > first) {
      const int l = lead.back();
      double dd = 0, kk = 0, ll = 0;
      for (int c = 0; c < 3; ++c) {
        const double a = qcart[3 * k + c], b = qcart[3 * l + c];
        dd += (a - b) * (a - b);
        kk += a * a;
        ll += b * b;
      }
      const double d = sqrt(dd);
      join = k - l < kmax && d <= dist && d <= rel * sqrt(std::min(kk, ll));
    }
    if (!join) lead.push_back(k);
    fmap[k] = f0 + (int)(lead.size() - first) - 1;
  }
  return (int)(lead.size() - first);
}

ClusterPlan cluster_plan(const double* theta, int nk, int s, const int* sel, int nsel, double dtol) {
  ClusterPlan p;
  p.lo.assign((size_t)nk * nsel, 0);
  p.hi.assign((size_t)nk * nsel, 0);
  std::vector<char> use(s, 0);
  for (int j = 0; j < nsel; ++j) use[sel[j]] = 1;
  auto th = [&](int k, int i) { return theta[(size_t)k * s + i]; };
  auto om = [&](int k, int i) { return sqrt(std::max(th(k, i), 0.0)); };
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nsel; ++j) {
      int l = sel[j], h = sel[j];
      if (dtol > 0 && th(k, sel[j]) > 0) {
        while (l > 0 && om(k, l) - om(k, l - 1) < dtol * om(k, l)) --l;
        while (h + 1 < s && om(k, h + 1) - om(k, h) < dtol * om(k, h + 1)) ++h;
      }
      p.lo[(size_t)k * nsel + j] = l;
      p.hi[(size_t)k * nsel + j] = h;
      if (h > l) {
        ++p.ndeg;
        for (int i = l; i <= h; ++i) use[i] = 1;
      }
    }
  if (p.ndeg == 0) {
    p.ext.assign(sel, sel + nsel);
    return p;
  }
  for (int i = 0; i < s; ++i)
    if (use[i]) p.ext.push_back(i);
  const size_t next = p.ext.size();
  p.coef.assign((size_t)nk * nsel * next, 0.0);
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nsel; ++j) {
      const int l = p.lo[(size_t)k * nsel + j], h = p.hi[(size_t)k * nsel + j];
      for (size_t t = 0; t < next; ++t)
        if (p.ext[t] >= l && p.ext[t] <= h) p.coef[((size_t)k * nsel + j) * next + t] = 1.0 / (h - l + 1);
    }
  return p;
}

}  // namespace phx_host

extern "C" {

int phx_validate(const phx_cell* cell, const double* rho, int nk, const double* q, int nbands, int nsens,
                 const int* band_no, char* msg, int msglen) {
  const char* e = phx_host::check_cell(cell);
  if (!e && rho) e = phx_host::check_rho(rho, (long)cell->nv * cell->nv * cell->nv);
  if (!e && (q || nk)) e = phx_host::check_q(q, nk);
  if (!e && (nbands || nsens)) e = phx_host::check_bands(cell, nbands, nsens, band_no, 0);
  if (msg && msglen > 0) {
    strncpy(msg, e ? e : "", (size_t)msglen - 1);
    msg[msglen - 1] = 0;
  }
  return e ? PHX_EINVAL : PHX_OK;
}

int phx_kpath(phx_lattice lattice, const char* path, int nk, double* q_out) {
  return phx_host::kpath(lattice, path, nk, q_out);
}

int phx_projection_size(const phx_projection* p, long* ndesign) {
  if (!ndesign) return PHX_EINVAL;
  return phx_host::projection_shape(p, ndesign) ? PHX_EINVAL : PHX_OK;
}

}  // extern "C"
