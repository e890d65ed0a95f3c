// Driver for the host module of the library (csrc/host.cpp), built with the host compiler
// under the address and undefined-behaviour sanitizers by test_host_sanitize.py.  Each mode
// reads its cases from stdin and prints the results as plain numbers, one case per line.
//
//   kpath:  "lattice nk path" ("-" = default path)  ->  "rc q0 q1 ..."
//   plan:   "nk s nsel dtol theta... sel..."        ->  "ndeg | lo... | hi... | ext... | coef..."
//   groups: "nk kmax dist rel f0 qcart... which..." ->  "ngroups | fmap... | lead..."
//   cell:   "lattice a M nv rho0 E0 nu0 rho1 E1 nu1 simp nb block nsens band..." -> "cell-msg | bands-msg"
//   proj:   "nv spacing radius beta octant"         ->  "ndesign-or--1 | msg"
//   size:   "nk mem_gb n3 Np nb N prec precond block" -> "s per kc"
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "../paper_1603_06855_amd/csrc/phx_host.h"

static const char* msg(const char* e) { return e ? e : "ok"; }

// strtod reads "nan" and "inf", which operator>> does not
static double num(std::istream& in) {
  std::string t;
  in >> t;
  return strtod(t.c_str(), nullptr);
}

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  const std::string mode = argv[1];
  std::string line;
  while (std::getline(std::cin, line)) {
    if (line.empty()) continue;
    std::istringstream in(line);
    if (mode == "kpath") {
      int lat, nk;
      std::string path;
      in >> lat >> nk >> path;
      std::vector<double> q(3L * (nk > 0 ? nk : 1), -7.0);
      const int rc = phx_kpath((phx_lattice)lat, path == "-" ? nullptr : path.c_str(), nk, q.data());
      printf("%d", rc);
      if (rc == PHX_OK)
        for (double v : q) printf(" %.17g", v);
      printf("\n");
    } else if (mode == "plan") {
      int nk, s, nsel;
      double dtol;
      in >> nk >> s >> nsel;
      dtol = num(in);
      std::vector<double> th((size_t)nk * s);
      std::vector<int> sel(nsel);
      for (auto& v : th) v = num(in);
      for (auto& v : sel) in >> v;
      const phx_host::ClusterPlan p = phx_host::cluster_plan(th.data(), nk, s, sel.data(), nsel, dtol);
      printf("%ld |", p.ndeg);
      for (int v : p.lo) printf(" %d", v);
      printf(" |");
      for (int v : p.hi) printf(" %d", v);
      printf(" |");
      for (int v : p.ext) printf(" %d", v);
      printf(" |");
      for (double v : p.coef) printf(" %.17g", v);
      printf("\n");
    } else if (mode == "groups") {
      int nk, kmax, f0;
      double dist, rel;
      in >> nk >> kmax;
      dist = num(in);
      rel = num(in);
      in >> f0;
      std::vector<double> qc(3L * nk);
      std::vector<char> which(nk);
      for (auto& v : qc) v = num(in);
      for (auto& v : which) {
        int w;
        in >> w;
        v = (char)w;
      }
      std::vector<int> fmap(nk, -1), lead;
      const int ng = phx_host::share_groups(qc.data(), nk, which.data(), kmax, dist, rel, f0, fmap.data(), lead);
      printf("%d |", ng);
      for (int v : fmap) printf(" %d", v);
      printf(" |");
      for (int v : lead) printf(" %d", v);
      printf("\n");
    } else if (mode == "cell") {
      phx_cell c;
      memset(&c, 0, sizeof c);
      int lat, nb, block, nsens;
      in >> lat;
      c.a = num(in);
      in >> c.M >> c.nv;
      for (phx_material* m : {&c.phase0, &c.phase1}) {
        m->density = num(in);
        m->youngs = num(in);
        m->poisson = num(in);
      }
      c.simp_p = num(in);
      in >> nb >> block >> nsens;
      c.lattice = (phx_lattice)lat;
      std::vector<int> band(nsens > 0 ? nsens : 0);
      for (auto& v : band) in >> v;
      const char* ec = phx_host::check_cell(&c);
      const char* eb = ec ? nullptr : phx_host::check_bands(&c, nb, nsens, band.empty() ? nullptr : band.data(), block);
      printf("%s | %s\n", msg(ec), msg(eb));
    } else if (mode == "proj") {
      phx_projection p;
      memset(&p, 0, sizeof p);
      in >> p.nv >> p.spacing;
      p.radius = num(in);
      p.beta = num(in);
      in >> p.octant;
      long nd = -1;
      const char* e = phx_host::check_projection(&p, &nd);
      printf("%ld | %s\n", e ? -1L : nd, msg(e));
    } else if (mode == "size") {
      int nk, nb, N, prec, precond, block;
      double mem_gb;
      long n3, Np;
      in >> nk;
      mem_gb = num(in);
      in >> n3 >> Np >> nb >> N >> prec >> precond >> block;
      const int s = phx_host::choose_block(block, nb, N);
      const long per = phx_host::per_k_bytes(n3, Np, s, prec, precond);
      printf("%d %ld %d\n", s, per, phx_host::chunk_size(nk, mem_gb, per));
    } else {
      return 2;
    }
    if (in.fail()) return 3;  // a malformed case line
  }
  return 0;
}
