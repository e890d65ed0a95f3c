// Host runtime and C ABI of the phx library: argument validation,
// non-dimensionalisation, device workspaces, the per-design precompute and the
// batched block eigensolver over k-chunks, and the adjoint.
//
// Eigensolver (per k-chunk, all k in lock-step, every step a batched kernel):
//   A(k) = K(k) + sigma Omega is assembled and Cholesky-factored (FP64 or FP32);
//   X holds s >= nbands + guard search vectors, started from plane-wave unit
//   vectors of the smallest |K_p|.  Each iteration forms the basis S = [X W P]
//   (W: preconditioned residuals A^{-1} R, P: previous search direction, LOBPCG),
//   Omega-orthonormalises it twice (CholQR2 with column dropping), performs
//   Rayleigh-Ritz with K applied in FP64 without forming it (the k-independent
//   inverse compliance channels act on all k of the chunk in one GEMM), and
//   stops when every wanted band's relative residual is below tolerance.
#include <math.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/phx.h"
#include "phx_host.h"
#include "phx_internal.h"
#include "phx_physics.h"

using namespace phx;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Opts {
  double tol[2] = {1e-8, 1e-6};
  int maxit = 60;
  int block = 0;
  double shift = 0.02;
  // Omega-CholQR drops a column whose squared orthogonal part falls below drop times its
  // squared norm: kept columns are amplified by at most drop^-1/2 = 1e4, so the rounding
  // carried by the basis and its K / Omega images stays far below the FP64 tolerances
  // (with 1e-12, 1e6-fold amplification let the images of nearly dependent columns
  // drift until the iteration diverged on sharp high-contrast inclusions).
  double drop = 1e-8;
  double mem_gb = 64.0;
  int coarse = 1;            // start orders M >= 4 from the order M-2 Ritz vectors
  double coarse_tol = 1e-3;  // residual tolerance of that coarse solve
  int coarse_drop = 2;       // the coarse start's order: M - coarse_drop (at least 1)
  int streams = 4;           // designs solved concurrently by the batched call
  int rr_fused = 2;          // 1: second orthonormalisation folded into Rayleigh-Ritz; 2: both
  int small_eig = 1;         // eigensolver of the folded Rayleigh-Ritz problem: 0 Jacobi, 1 tridiagonal
  int sbinv = 1;             // 1: preconditioner solves through explicit super-block inverses
  int kskip = 1;             // 1: k-points whose wanted bands have converged skip later iterations
  int kshare = 2;            // at most this many consecutive k-points share one preconditioner factor
  double kshare_dist = 0.15; // ... if within this Cartesian distance (cycles per a) of the group's first
  double kshare_rel = 0.5;   // ... and within this fraction of the shorter of the two wave vectors
  int spin_wait = 0;         // 1: the per-iteration host wait spins (hipStreamSynchronize)
  int omega_conv = 1;        // 1: Omega_s X as a convolution (M <= 5); 0: the dense real operator
  double guard_lock = 1000;  // guard columns (beyond the wanted bands) lock below guard_lock x tol
  int zskip = 1;             // 1: the fused Rayleigh-Ritz step skips loading soft-locked (zero) columns
  int gram_split = 0;        // K-split of the Gram products (0: min(16, 3Np / 256))
  int kstreams = 1;          // single-design device calls: k-point ranges on this many streams
  double degen_tol = 1e-8;   // bands closer than this (relative, in omega) form one degenerate cluster
  double mem_limit_gb = 0;   // cap on the device workspace a context may hold (0: none)
  int precond = 2;           // 0: Cholesky of the pencil K + sigma Omega; 1: its 3 x 3 per-wave diagonal
                             // blocks; 2: the blocks until they stall, then the pencil
  int stall_its = 8;         // precond 2: a k-point stalls when its residual falls less than tenfold in this many iterations
};

struct Stats {
  int iters = 0, chunks = 0, block = 0, kchunk = 0;
  int rr_sweeps = 0;  // most Jacobi sweeps any k needed in a Rayleigh-Ritz step of the last solve
  int coarse_iters = 0;  // eigensolver iterations of the coarse start (slowest chunk)
  long k_conv_iters = 0, k_count = 0;  // sum over k of the iteration at which k converged
  long factors = 0;                     // preconditioner factorisations (order M solves)
  long degen = 0;                       // (k, requested band) entries inside a degenerate cluster
  int enomem_retries = 0;               // k-chunks retried with half as many k-points after ENOMEM
  int precond_switches = 0;             // k-points (of order-M and coarse solves) moved from Jacobi to the pencil
};

// Kernel-class timing with HIP events recorded on the context stream.
enum RtClass {
  PROF_ASSEMBLE = phx::PROF_NCLASS_DENSE,
  PROF_APPLY,     // strain and force (pointwise parts of the matrix-free K X)
  PROF_OP_GEMM,   // the k-shared operator products (Dm, Bm, Omega_s, real in the paired basis)
  PROF_GRAM,
  PROF_SMALL,
  PROF_UPDATE,
  PROF_RESIDUAL,
  PROF_ADJOINT,
  PROF_OP_CONV,   // Omega_s X as a convolution (omega_conv_kernel)
  PROF_NCLASS
};
const char* const PROF_NAMES[PROF_NCLASS] = {"potrf_diag", "panel",      "herk",  "trsm_diag", "trsm_update",
                                             "solve_upd",  "solve_diag", "sbinv", "assemble",  "apply",
                                             "op_gemm",    "gram",      "small", "update",    "residual",
                                             "adjoint",    "op_conv"};

struct PendKernel {
  int cls;
  double flops, bytes;
  bool set;
};

struct ProfAcc {
  double ms = 0, flops = 0, bytes = 0;
  long count = 0;
};

struct Profiler {
  bool on = false;
  bool stages = true;  // false: only the launches that record their own kernel events
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  struct Pend {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
  };
  std::vector<Pend> pend;
  hipEvent_t open = nullptr;
  ProfAcc acc[PROF_NCLASS];
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  void begin(int cls) {
    if (!on || !stages) return;
    open = get();
    if (open) (void)hipEventRecord(open, st);
  }
  // Two events for one kernel launch to record at the kernel's start and end; the
  // measurement is registered now and read at the next flush.
  void kernel_events(int cls, double flops, double bytes, hipEvent_t* a, hipEvent_t* b) {
    *a = *b = nullptr;
    if (!on) return;
    hipEvent_t e0 = get(), e1 = get();
    if (!e0 || !e1) return;
    pend.push_back({cls, e0, e1, flops, bytes});
    *a = e0;
    *b = e1;
  }
  void end(int cls, double flops, double bytes) {
    if (!on || !open) return;
    hipEvent_t b = get();
    if (!b) return;
    (void)hipEventRecord(b, st);
    pend.push_back({cls, open, b, flops, bytes});
    open = nullptr;
  }
  // Call after the stream has been synchronised.
  void flush() {
    for (auto& p : pend) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        acc[p.cls].ms += ms;
        acc[p.cls].flops += p.flops;
        acc[p.cls].bytes += p.bytes;
        acc[p.cls].count += 1;
      }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pend.clear();
  }
  void reset() {
    for (auto& a : acc) a = ProfAcc();
  }
  ~Profiler() {
    for (auto& p : pend) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

void hook_begin(void* u, int cls) { ((Profiler*)u)->begin(cls); }
void hook_end(void* u, int cls, double f, double b) { ((Profiler*)u)->end(cls, f, b); }
void hook_kev(void* u, int cls, double f, double b, hipEvent_t* e0, hipEvent_t* e1) {
  ((Profiler*)u)->kernel_events(cls, f, b, e0, e1);
}

// Device scratch of the allocation-free projection adjoint (phx_project_adjoint_dev_noalloc):
// the per-element coefficients of one call, nv^3 doubles, nv <= 64 (2 MiB).  Every GPU the
// library runs on holds its own copy until the process ends; host code reaches it only
// through the per-device address taken at context creation (the array's name is a host
// stand-in, not a device address).
constexpr long NOALLOC_SCRATCH_DOUBLES = 64L * 64 * 64;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_addr;  // device -> address of its scratch

// Takes the current device's address of the scratch array once per device.
int scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr.count(device)) return PHX_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PHX_EHIP;
  g_scratch_addr[device] = (double*)ptr;
  return PHX_OK;
}

double* scratch_addr(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  return it == g_scratch_addr.end() ? nullptr : it->second;
}

}  // namespace

// Statistics of several solves: the largest of the per-solve maxima, the sums of counts.
void merge_stats(Stats& into, const Stats& s) {
  into.iters = std::max(into.iters, s.iters);
  into.rr_sweeps = std::max(into.rr_sweeps, s.rr_sweeps);
  into.coarse_iters = std::max(into.coarse_iters, s.coarse_iters);
  into.k_conv_iters += s.k_conv_iters;
  into.factors += s.factors;
  into.k_count += s.k_count;
  into.chunks += s.chunks;
  into.block = std::max(into.block, s.block);
  into.kchunk = std::max(into.kchunk, s.kchunk);
  into.degen += s.degen;
  into.enomem_retries += s.enomem_retries;
  into.precond_switches += s.precond_switches;
}

struct phx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = true;
  std::string err;
  std::map<std::string, DevBuf> bufs;
  size_t mem_used = 0;  // bytes held in bufs
  int* dflag = nullptr;
  Opts opt;
  Stats stats;
  bool trace = false;
  Profiler prof;
  PendKernel pk{0, 0, 0, false};  // timing request for the next GEMM launch
  hipEvent_t wait_ev = nullptr;   // blocking-sync event of the per-iteration host wait
  void* hpin = nullptr;           // pinned host staging of the per-iteration read-backs
  size_t hpin_bytes = 0;
  std::vector<phx_ctx*> workers;  // contexts (own stream and workspaces) of the batched call
  phx::ProfHook hook{hook_begin, hook_end, hook_kev, nullptr};
  const phx::ProfHook* hk() {
    hook.user = &prof;
    prof.st = stream;
    return prof.on ? &hook : nullptr;
  }
};

#define PROF_BEGIN(c) ctx->prof.begin(c)
#define PROF_END(c, f, b) ctx->prof.end((c), (f), (b))
// The next GEMM launch on ctx is timed by events recorded at its kernel's start and end.
#define PROF_KERNEL(c, f, b) ctx->pk = PendKernel{(c), (f), (b), true}

namespace {

struct Fail {
  int code;
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);                    \
      throw Fail{e_ == hipErrorOutOfMemory ? PHX_ENOMEM : PHX_EHIP};                   \
    }                                                                                  \
  } while (0)

#define KCHK(expr)                                                                     \
  do {                                                                                 \
    int e_ = (int)(expr);                                                              \
    if (e_) {                                                                          \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString((hipError_t)e_);        \
      throw Fail{PHX_EHIP};                                                            \
    }                                                                                  \
  } while (0)

[[noreturn]] void fail(phx_ctx* ctx, int code, const std::string& msg) {
  ctx->err = msg;
  throw Fail{code};
}

template <typename T>
T* dbuf(phx_ctx* ctx, const std::string& name, size_t count) {
  DevBuf& b = ctx->bufs[name];
  const size_t need = std::max<size_t>(count * sizeof(T), 256);
  if (b.bytes < need) {
    const double lim = ctx->opt.mem_limit_gb * 1073741824.0;
    if (lim > 0 && (double)(ctx->mem_used - b.bytes + need) > lim) {
      ctx->err = "workspace " + name + " (" + std::to_string(need) + " bytes) would exceed mem_limit_gb";
      throw Fail{PHX_ENOMEM};
    }
    if (b.p) HIPCHK(hipFree(b.p));
    ctx->mem_used -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipMalloc(&b.p, need);
    if (e != hipSuccess) {
      b.p = nullptr;
      ctx->err = "hipMalloc(" + name + ", " + std::to_string(need) + " bytes): " + hipGetErrorString(e);
      throw Fail{PHX_ENOMEM};
    }
    b.bytes = need;
    ctx->mem_used += need;
  }
  return (T*)b.p;
}

// Frees every workspace except the per-design data (names with a design tag) and the
// sensitivity output of the call in progress; after a device wait, so no queued kernel
// still reads them.
void release_workspaces(phx_ctx* ctx) {
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (auto it = ctx->bufs.begin(); it != ctx->bufs.end();) {
    const std::string& n = it->first;
    if (n.rfind("d0:", 0) == 0 || n.rfind("c0:", 0) == 0 || n == "sens") {
      ++it;
      continue;
    }
    if (it->second.p) HIPCHK(hipFree(it->second.p));
    ctx->mem_used -= it->second.bytes;
    it = ctx->bufs.erase(it);
  }
}

// Pinned host staging area of at least `bytes` (grow-only, one per context).
void* hbuf(phx_ctx* ctx, size_t bytes) {
  if (ctx->hpin_bytes < bytes) {
    if (ctx->hpin) HIPCHK(hipHostFree(ctx->hpin));
    ctx->hpin = nullptr;
    ctx->hpin_bytes = 0;
    if (hipHostMalloc(&ctx->hpin, bytes, hipHostMallocDefault) != hipSuccess) {
      ctx->hpin = nullptr;
      ctx->err = "hipHostMalloc(" + std::to_string(bytes) + " bytes) failed";
      throw Fail{PHX_ENOMEM};
    }
    ctx->hpin_bytes = bytes;
  }
  return ctx->hpin;
}

// Host wait for everything queued on st: a blocking-sync event, so that the waiting
// thread sleeps instead of spinning on a core the other design streams' threads need
// to launch their work (option spin_wait = 1: hipStreamSynchronize).
void wait_stream(phx_ctx* ctx, hipStream_t st) {
  if (ctx->opt.spin_wait) {
    HIPCHK(hipStreamSynchronize(st));
    return;
  }
  HIPCHK(hipEventRecord(ctx->wait_ev, st));
  HIPCHK(hipEventSynchronize(ctx->wait_ev));
}

using phx_host::prim_rows;
using phx_host::reciprocal;

void check_cell(phx_ctx* ctx, const phx_cell* c) {
  if (const char* e = phx_host::check_cell(c)) fail(ctx, PHX_EINVAL, e);
}

void check_rho(phx_ctx* ctx, const double* rho, long n) {
  if (const char* e = phx_host::check_rho(rho, n)) fail(ctx, PHX_EINVAL, e);
}

void check_q(phx_ctx* ctx, const double* q, int nk) {
  if (const char* e = phx_host::check_q(q, nk)) fail(ctx, PHX_EINVAL, e);
}

// ---------------------------------------------------------------------------
// Per-design precompute (k-independent): fields, Fourier tables, Toeplitz
// gathers, and the inverse compliance channels.
// ---------------------------------------------------------------------------
struct Design {
  phx_cell cell;
  int M, N, Np, n3, nv;
  long nvox;
  double V, v, c2, lscale, sigma, dens_min;
  MaterialND mat;
  Recip rec;
  std::string tag;
  double* rho_d = nullptr;
  double2* tab = nullptr;  // 3 x (4M+1)^3
  double2* Os = nullptr;   // Np x Np
  double2* Dm = nullptr;   // Pv^{-1} - Pd^{-1}
  double2* Bm = nullptr;   // Pd^{-1}
  // Phi_vol^-1 = Dm + Bm, Bm = Phi_dev^-1 and Os in the basis pairing each wave n_p with -n_p
  // (launch_realify), where they are real: the eigensolver's vectors live in that basis
  double* Vr = nullptr;
  double* Br = nullptr;
  double* Or = nullptr;
  double2* Ch = nullptr;  // the density table transformed along n2, n3 (launch_omega_table), M <= 5
};

MaterialND nondim(const phx_cell& c) {
  const double E0 = c.phase0.youngs, r0 = c.phase0.density;
  auto ch = [&](const phx_material& m, double& dens, double& cv, double& cd) {
    const double E = m.youngs / E0, nu = m.poisson;
    const double K = E / (3.0 * (1.0 - 2.0 * nu)), G = E / (2.0 * (1.0 + nu));
    dens = m.density / r0;
    cv = 1.0 / (3.0 * K);
    cd = 1.0 / (2.0 * G);
  };
  double d0, v0, s0, d1, v1, s1;
  ch(c.phase0, d0, v0, s0);
  ch(c.phase1, d1, v1, s1);
  MaterialND m;
  m.p = c.simp_p;
  m.dens0 = d0; m.ddens = d1 - d0;
  m.cvol0 = v0; m.dcvol = v1 - v0;
  m.cdev0 = s0; m.dcdev = s1 - s0;
  return m;
}

void setup_geometry(const phx_cell& cell, Design& d) {
  d.cell = cell;
  d.M = cell.M;
  const int L = 2 * cell.M + 1;
  d.N = L * L * L;
  d.Np = (d.N + 63) / 64 * 64;
  d.n3 = 3 * d.Np;
  d.nv = cell.nv;
  d.nvox = (long)cell.nv * cell.nv * cell.nv;
  double A[3][3], T[3][3];
  prim_rows(cell.lattice, A);
  d.V = reciprocal(A, T);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) d.rec.t[i][j] = T[i][j];
  d.v = d.V / (double)d.nvox;
  d.c2 = (2.0 * M_PI * d.V) * (2.0 * M_PI * d.V);
  d.lscale = cell.phase0.youngs / (cell.phase0.density * cell.a * cell.a);
  d.mat = nondim(cell);
}

// rho_host: the design on the host (used for the shift scale and bounds);
// rho_dev: the same design already on the device, or NULL to upload.
void setup_design(phx_ctx* ctx, const phx_cell& cell, const double* rho_host, const double* rho_dev, Design& d,
                  const std::string& tag) {
  setup_geometry(cell, d);
  d.tag = tag;
  hipStream_t st = ctx->stream;
  // shift scale and the density lower bound from the host copy
  double wsum = 0;
  for (long e = 0; e < d.nvox; ++e) wsum += pow(rho_host[e], cell.simp_p);
  const double wbar = wsum / d.nvox;
  double dens_mean = d.mat.dens0 + wbar * d.mat.ddens;
  double cdev_mean = d.mat.cdev0 + wbar * d.mat.dcdev;
  double bmin = 1e300;
  for (int j = 0; j < 3; ++j)
    bmin = std::min(bmin, d.rec.t[j][0] * d.rec.t[j][0] + d.rec.t[j][1] * d.rec.t[j][1] + d.rec.t[j][2] * d.rec.t[j][2]);
  const double lam_scale = 4.0 * M_PI * M_PI * bmin * (1.0 / (2.0 * cdev_mean)) / dens_mean;
  d.sigma = ctx->opt.shift * lam_scale;
  {
    double lo = 1e300;
    for (long e = 0; e < d.nvox; ++e) lo = std::min(lo, d.mat.dens0 + pow(rho_host[e], cell.simp_p) * d.mat.ddens);
    d.dens_min = lo;
  }

  if (rho_dev) {
    d.rho_d = const_cast<double*>(rho_dev);
  } else {
    d.rho_d = dbuf<double>(ctx, tag + "rho", d.nvox);
    HIPCHK(hipMemcpyAsync(d.rho_d, rho_host, d.nvox * sizeof(double), hipMemcpyHostToDevice, st));
  }
  const int M2 = 2 * d.M, L2 = 2 * M2 + 1;
  double* F = dbuf<double>(ctx, "F", 3 * d.nvox);
  double2* G1 = dbuf<double2>(ctx, "G1", 3L * d.nv * d.nv * L2);
  double2* G2 = dbuf<double2>(ctx, "G2", 3L * d.nv * L2 * L2);
  d.tab = dbuf<double2>(ctx, tag + "tab", 3L * L2 * L2 * L2);
  launch_fields(d.rho_d, (int)d.nvox, d.mat, F, st);
  launch_dft(F, d.nv, d.M, d.v, G1, G2, d.tab, st);
  KCHK(hipGetLastError());
  if (d.M <= OMEGA_CONV_MAX_M) {
    d.Ch = dbuf<double2>(ctx, tag + "och", (size_t)L2 * L2 * L2);
    launch_omega_table(d.tab, d.M, d.Ch, st);
    KCHK(hipGetLastError());
  }

  const long NN = (long)d.Np * d.Np;
  double2* ops = dbuf<double2>(ctx, tag + "ops", 3 * NN);  // Os, Pv, Pd -> Os, factors
  double2* inv = dbuf<double2>(ctx, tag + "inv", 2 * NN);  // Pv^{-1} - Pd^{-1}, Pd^{-1}
  double2* work = dbuf<double2>(ctx, "phi_work", 2 * NN);
  double2* dinv = dbuf<double2>(ctx, "phi_dinv", 2L * (d.Np / 64) * 4096);
  launch_gather(d.tab, d.M, d.N, d.Np, ops, st);
  KCHK(hipGetLastError());
  HIPCHK(hipMemsetAsync(ctx->dflag, 0, sizeof(int), st));
  KCHK(potrf_batched<double>(ops + NN, d.Np, d.Np, NN, 2, dinv, (long)(d.Np / 64) * 4096, ctx->dflag, st));
  launch_identity(inv, d.Np, 2, st);
  KCHK(potrs_batched<double>(ops + NN, d.Np, d.Np, NN, 2, dinv, (long)(d.Np / 64) * 4096, inv, d.Np, NN, work,
                             d.Np, NN, d.Np, st));
  launch_split_inverse(inv, inv + NN, NN, st);
  KCHK(hipGetLastError());
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, ctx->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (flag) fail(ctx, PHX_ENOTPD, "compliance Fourier matrix is not positive definite");
  d.Os = ops;
  d.Dm = inv;
  d.Bm = inv + NN;
  // the operators in the basis where they are real: each product with a complex block takes
  // two real products instead of three
  d.Vr = dbuf<double>(ctx, tag + "opr", 3 * NN);
  d.Br = d.Vr + NN;
  d.Or = d.Vr + 2 * NN;
  launch_realify(d.Dm, d.N, d.Np, d.Vr, st, d.Bm);
  launch_realify(d.Bm, d.N, d.Np, d.Br, st);
  launch_realify(d.Os, d.N, d.Np, d.Or, st);
  KCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Eigensolver over one chunk of k-points.
// ---------------------------------------------------------------------------
struct ChunkOut {
  std::vector<double> theta;  // nk x s (non-dimensional lambda)
  std::vector<double> rnorm;  // nk x s
  std::vector<double> rn;     // nk x s
  int iters = 0;
  bool converged = false;
};

// Columns of the eigensolver basis known to be zero (GemmArgs::zrn).
struct ZeroCols {
  const double* rn;
  double tol, gtol;
  int s, nb, first;
};

struct Solver {
  phx_ctx* ctx;
  Design* d;
  int nk, nb, s, m, prec;
  long n3, sBig;
  double2* Big;
  double* Kv;
  double* sigma_d;
  double2 *Y, *Tr, *Zy, *Zt;
  double2 *G, *Gpart, *C0, *Cr;
  double2 *G2, *G2part, *Cp;
  int* keep;
  int* sweeps;
  double *theta, *rn, *rnorm;
  void* A;     // nk x n3 x n3 (prec)
  void* Dinv;  // nk x n3/64 x 4096 (prec)
  void* SBinv; // nk x nsb x WS^2 inverses of the factor's diagonal super-blocks, or NULL
  int* kact;   // per k: 1 while a wanted band of that k-point has not met the tolerance
  int* kfar;   // per k: active and not yet near convergence (folded Rayleigh-Ritz)
  int* knear;  // per k: active and near convergence (explicit re-orthonormalisation, images recomputed)
  int* lact;   // the k-points of kact, kfar and knear listed in ascending order (3 nk ints in all)
  int* lfar;
  int* lnear;
  int* fmap;   // per k: index of its preconditioner factor (NULL: its own)
  int nact;    // active k-points (host count of kact)
  int nfar, nnear;
  int* kjac;   // per k: active and preconditioned by block Jacobi
  int* kpen;   // per k: active and preconditioned by its pencil factor
  int njac, npen;
  int nf, fcap;  // pencil factors built so far, and the capacity of the factor arrays
  void* Rp;    // nk x n3 x s
  void* Zp;
  int ksplit;
  // the soft-locked columns of the current basis, whose W and P parts and images the last
  // residual kernel zeroed (rn, the thresholds it used), or before the first step all of W
  // and P; the fused Rayleigh-Ritz step's Gram product and update skip loading them
  ZeroCols zc{nullptr, 0, 0, 0, 0, 0};
};

template <typename R>
void gemm(phx_ctx* ctx, int opa, int opb, int M, int N, int K, int batch, const C_t<R>* A, long lda, long sA, int dA,
          const C_t<R>* B, long ldb, long sB, int dB, C_t<R>* Cm, long ldc, long sC, C_t<R> alpha, C_t<R> beta,
          int ksplit = 1, C_t<R>* Cpart = nullptr, const int* kact = nullptr, int kdiv = 1, int csplit = 0,
          int cgap = 0, const int* bidx = nullptr, int nbat = 0, int tiled = 0, const ZeroCols* zc = nullptr) {
  GemmArgs<R> g{};
  if (zc) {
    g.zrn = zc->rn;
    g.ztol = zc->tol;
    g.zgtol = zc->gtol;
    g.zs = zc->s;
    g.znb = zc->nb;
    g.zfirst = zc->first;
  }
  if (ctx->pk.set) {
    ctx->prof.kernel_events(ctx->pk.cls, ctx->pk.flops, ctx->pk.bytes, &g.ev0, &g.ev1);
    ctx->pk.set = false;
  }
  g.csplit = csplit;
  g.cgap = cgap;
  g.kact = kact;
  g.bidx = bidx;
  g.nbat = nbat;
  g.tiled = tiled;
  g.kdiv = kdiv;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.A = A; g.lda = lda; g.sA = sA; g.dA = dA;
  g.B = B; g.ldb = ldb; g.sB = sB; g.dB = dB;
  g.Cm = Cm; g.ldc = ldc; g.sC = sC; g.dC = 1;
  g.alpha = alpha; g.beta = beta;
  g.ksplit = ksplit; g.Cpart = Cpart;
  KCHK(zgemm<R>(g, opa, opb, ctx->stream));
}

const double2 ONE = {1.0, 0.0}, ZERO = {0.0, 0.0};

// K and Omega applied (FP64, matrix-free, paired basis) to ncol columns of the S block of
// Big starting at column c0; results to the same columns of the KS and OS blocks.
// msk (device, per k; NULL: sv.kact) selects the k-points, nm counts them and lst lists
// them (device, nm entries).  cl (optional, device): only the nc columns it lists
// (entries k * ncol + j) go through the operator products, and cm (device, per
// k * ncol + j) marks the same columns for the strain and force kernels; the images of the
// other columns are left as they are.
void apply_ops(Solver& sv, double2* Big, int c0, int ncol, const int* msk = nullptr, int nm = -1,
               const int* lst = nullptr, const int* cl = nullptr, int nc = 0, const int* cm = nullptr) {
  phx_ctx* ctx = sv.ctx;
  Design& d = *sv.d;
  hipStream_t st = ctx->stream;
  const long n3 = sv.n3, m = sv.m;
  if (!msk) {
    msk = sv.kact;
    nm = sv.nact;
    lst = sv.lact;
  }
  if (nm <= 0) return;
  double2* X = Big + c0 * n3;
  const double Np = d.Np, nk = nm;  // algorithmic work counts the selected k-points only
  PROF_BEGIN(PROF_APPLY);
  // strain channels of the paired-basis columns, in the same basis
  launch_strain(X, n3, sv.sBig, sv.Kv, d.Np, ncol, sv.nk, sv.Y, sv.Tr, st, msk, d.N, cl ? cm : nullptr);
  const double ncv = cl ? (double)nc : nk * ncol;  // vectors through the operators
  PROF_END(PROF_APPLY, 0, 16.0 * ncv * (3.0 + 6.0) * Np);
  KCHK(hipGetLastError());
  // The real operator products in one launch, over the listed k-points: the deviatoric
  // compliance Bm times the five deviatoric strain channels, the volumetric compliance
  // Phi_vol^-1 times the volumetric channel and, unless it is applied as a convolution
  // (option omega_conv, M <= 5), Omega_s times the columns (one column per vector: those
  // of the listed k-points form one product); six or nine operator columns per vector.
  // 4 Np^2 flops per complex column (two real products); each operator (8 B per entry)
  // read once, each block read and written once.
  const bool conv = ctx->opt.omega_conv && d.Ch;
  const int ny = 5 * ncol;
  OpArgs a{};
  a.M = a.K = d.Np;
  a.lda = d.Np;
  // (each product over the listed k-points' columns, or the listed vectors' columns, packed
  // side by side)
  const long sy = (long)d.Np * ny, st1 = (long)d.Np * ncol;
  double2* OX = Big + (2 * m + c0) * n3;
  OpSeg sb, so, sw;
  if (cl) {
    sb = OpSeg{d.Br, sv.Y, sv.Zy, (long)d.Np, sy, (long)d.Np, sy, 0, nc, 5, cl, ncol};
    so = OpSeg{d.Or, X, OX, (long)d.Np, sv.sBig, (long)d.Np, sv.sBig, 0, nc, 3, cl, ncol};
    sw = OpSeg{d.Vr, sv.Tr, sv.Zt, (long)d.Np, st1, (long)d.Np, st1, 0, nc, 1, cl, ncol};
  } else {
    sb = OpSeg{d.Br, sv.Y, sv.Zy, (long)d.Np, sy, (long)d.Np, sy, 0, nm, ny, lst, 1};
    so = OpSeg{d.Or, X, OX, (long)d.Np, sv.sBig, (long)d.Np, sv.sBig, 0, nm, 3 * ncol, lst, 1};
    sw = OpSeg{d.Vr, sv.Tr, sv.Zt, (long)d.Np, st1, (long)d.Np, st1, 0, nm, ncol, lst, 1};
  }
  a.seg[0] = sb;
  if (conv) {
    a.nseg = 2;
    a.seg[1] = sw;
  } else {
    a.nseg = 3;
    a.seg[1] = so;
    a.seg[2] = sw;
  }
  const double nop = conv ? 6.0 : 9.0;
  PROF_KERNEL(PROF_OP_GEMM, 4.0 * Np * Np * nop * ncv, (double)a.nseg * 8.0 * Np * Np + 32.0 * Np * nop * ncv);
  if (ctx->pk.set) {
    ctx->prof.kernel_events(ctx->pk.cls, ctx->pk.flops, ctx->pk.bytes, &a.ev0, &a.ev1);
    ctx->pk.set = false;
  }
  KCHK(opgemm(a, st));
  if (conv) {
    // its own arithmetic per component column: the forward DFT lines (L^2 along n3, L L2
    // along n2, 16M^2 + 14M flops each), the Toeplitz lines (L2^2 of L^2 complex
    // multiply-adds) and the inverse lines (L L2 and L^2, 16M^2 + 16M flops each); the
    // column read and written once (16 B per complex)
    const double Md = d.M, L = 2 * Md + 1, L2 = 4 * Md + 1;
    const double fcol = (L * L + L * L2) * (16 * Md * Md + 14 * Md) + L2 * L2 * 8 * L * L +
                        (L * L2 + L * L) * (16 * Md * Md + 16 * Md);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ctx->prof.kernel_events(PROF_OP_CONV, 3.0 * ncv * fcol, 3.0 * ncv * 32.0 * d.N, &e0, &e1);
    launch_omega_conv(ConvCols{so.B, so.C, so.sB, so.ldb, so.nb, so.ncolk, so.kdiv, so.bidx}, d.M, d.Np, d.Ch, st,
                      e0, e1);
    KCHK(hipGetLastError());
  }
  PROF_BEGIN(PROF_APPLY);
  launch_force(sv.Zy, sv.Zt, sv.Kv, d.Np, ncol, sv.nk, d.c2, Big + (m + c0) * n3, n3, sv.sBig, st, msk, d.N,
               cl ? cm : nullptr);
  PROF_END(PROF_APPLY, 0, 16.0 * ncv * (6.0 + 3.0) * Np);
  KCHK(hipGetLastError());
}

// The k-point selection of one eigensolver step: a device mask and its host count.
struct Sel {
  const int* d;  // per-k mask
  int n;         // its count
  const int* l;  // the selected k-points, listed (n entries)
};

void gram(Solver& sv, double2* Big, int block, Sel k) {
  // G_k = S_k^H (block_k), block 1 = KS, 2 = OS
  phx_ctx* ctx = sv.ctx;
  const long n3 = sv.n3, m = sv.m;
  PROF_BEGIN(PROF_GRAM);
  gemm<double>(sv.ctx, 1, 0, m, m, n3, sv.nk, Big, n3, sv.sBig, 1, Big + block * m * n3, n3, sv.sBig, 1, sv.G, m,
               m * m, ONE, ZERO, sv.ksplit, sv.Gpart, k.d, 1, 0, 0, k.l, k.n);
  PROF_END(PROF_GRAM, 8.0 * m * m * 3.0 * sv.d->N * k.n, 16.0 * 2 * m * 3.0 * sv.d->N * k.n);
}

// Basis update in place, for every k and each of the blocks S, KS, Omega S (batch 3 nk,
// the k-point's coefficients shared by its three blocks): columns c0 .. c0 + ncol - 1 of
// the new block are the old block's columns a0 .. a0 + K - 1 times the K x ncol
// coefficients C, written from column c0 (with split > 0: output columns split .. are
// written split further right, the tall-skinny kernel's split store).  Every output row
// depends only on the same row of the old block, and every kernel this product can run
// on (N <= 64: the tall-skinny kernel, the few-right-hand-side kernel or one column tile
// of the tiled kernel) reads a row's whole K range before it writes that row, and no two
// workgroups share a row, so reading and writing the same array is safe.  Frozen
// k-points are skipped and keep their basis.
void update_in_place(Solver& sv, long a0, long ncol, long K, const double2* C, long sC, long c0, int split,
                     Sel k, const ZeroCols* zc = nullptr) {
  phx_ctx* ctx = sv.ctx;
  const long n3 = sv.n3, m = sv.m;
  if (ncol > 64 || K > 64) fail(ctx, PHX_EINVAL, "in-place basis update needs at most 64 columns");
  if (zc && a0 != 0) fail(ctx, PHX_EINVAL, "zero-column skipping needs the whole basis from column 0");
  gemm<double>(ctx, 0, 0, n3, ncol, K, 3 * sv.nk, sv.Big + a0 * n3, n3, n3 * m, 1, C, m, sC, 3, sv.Big + c0 * n3, n3,
               n3 * m, ONE, ZERO, 1, nullptr, k.d, 3, split, split, k.l, k.n, 0, zc);
}

void cholqr(Solver& sv, Sel k) {
  phx_ctx* ctx = sv.ctx;
  const long m = sv.m;
  gram(sv, sv.Big, 2, k);
  PROF_BEGIN(PROF_SMALL);
  launch_chol_drop(sv.G, m, sv.nk, ctx->opt.drop, sv.C0, sv.keep, ctx->stream, k.d);
  PROF_END(PROF_SMALL, 0, 0);
  KCHK(hipGetLastError());
  // [S | KS | OS] <- [S | KS | OS] C0 for every k: batch 3 nk, C0 shared by the three blocks
  // (in place: see update_in_place)
  PROF_BEGIN(PROF_UPDATE);
  update_in_place(sv, 0, m, m, sv.C0, m * m, 0, 0, k);
  PROF_END(PROF_UPDATE, 8.0 * 3 * 3.0 * sv.d->N * m * m * k.n, 16.0 * 2 * 3 * 3.0 * sv.d->N * m * k.n);
}

void rayleigh_ritz(Solver& sv, Sel k) {
  phx_ctx* ctx = sv.ctx;
  const long m = sv.m, s = sv.s;
  gram(sv, sv.Big, 1, k);
  PROF_BEGIN(PROF_SMALL);
  launch_rr_eig(sv.G, sv.keep, m, s, sv.nk, sv.Cr, sv.theta, sv.sweeps, ctx->stream, k.d);
  PROF_END(PROF_SMALL, 0, 0);
  KCHK(hipGetLastError());
  // X <- [S] Cr ; P <- [W P] Cr[s:m]
  PROF_BEGIN(PROF_UPDATE);
  // In place (see update_in_place), X first: it reads the whole old basis and writes only
  // X, which the product for P does not read; P then reads W and the old P and writes P.
  update_in_place(sv, 0, s, m, sv.Cr, m * s, 0, 0, k);
  update_in_place(sv, s, s, m - s, sv.Cr + s, m * s, 2 * s, 0, k);
  PROF_END(PROF_UPDATE, 8.0 * 3 * 3.0 * sv.d->N * (2.0 * m - s) * s * k.n,
           16.0 * 3 * 3.0 * sv.d->N * (m + 2.0 * s) * k.n);
}

// Rayleigh-Ritz on the once-orthonormalised basis: both Gram matrices S^H [KS | Omega S]
// in one GEMM, the small kernel re-orthonormalises in the m x m space and solves the
// projected problem, and the Ritz vectors X and previous directions P are formed from
// the whole basis with the combined coefficients.
void rayleigh_ritz_fused(Solver& sv, Sel k) {
  phx_ctx* ctx = sv.ctx;
  const long n3 = sv.n3, m = sv.m, s = sv.s;
  PROF_BEGIN(PROF_GRAM);
  const ZeroCols* zc = sv.zc.rn ? &sv.zc : nullptr;
  gemm<double>(ctx, 1, 0, m, 2 * m, n3, sv.nk, sv.Big, n3, sv.sBig, 1, sv.Big + m * n3, n3, sv.sBig, 1, sv.G2, m,
               2 * m * m, ONE, ZERO, sv.ksplit, sv.G2part, k.d, 1, 0, 0, k.l, k.n, 0, zc);
  PROF_END(PROF_GRAM, 8.0 * m * 2 * m * 3.0 * sv.d->N * k.n, 16.0 * 3 * m * 3.0 * sv.d->N * k.n);
  PROF_BEGIN(PROF_SMALL);
  // coefficients of the new X and P side by side (m x 2s per k), so that one pass over
  // the basis produces both: columns 0..s-1 -> X, s..2s-1 -> P (basis columns 2s..3s-1)
  launch_rr_gen(sv.G2, m, s, sv.nk, ctx->opt.drop, sv.C0, sv.keep, sv.Cp, sv.Cp + m * s, sv.theta, sv.sweeps,
                ctx->stream, k.d, 2 * m * s, ctx->opt.small_eig);
  PROF_END(PROF_SMALL, 0, 0);
  KCHK(hipGetLastError());
  PROF_BEGIN(PROF_UPDATE);
  update_in_place(sv, 0, 2 * s, m, sv.Cp, 2 * m * s, 0, (int)s, k, zc);
  PROF_END(PROF_UPDATE, 8.0 * 3 * 3.0 * sv.d->N * 2.0 * m * s * k.n, 16.0 * 3 * 3.0 * sv.d->N * (m + 2.0 * s) * k.n);
}

template <typename R>
void precondition(Solver& sv) {
  phx_ctx* ctx = sv.ctx;
  const long n3 = sv.n3;
  if (sv.njac > 0) {  // block Jacobi: the per-wave 3 x 3 blocks, straight into W
    Design& d = *sv.d;
    PROF_BEGIN(PROF_APPLY);
    launch_jacobi<R>(d.Dm, d.Bm, d.Os, sv.Kv, d.N, d.Np, d.c2, sv.sigma_d, (const C_t<R>*)sv.Rp, n3 * sv.s, sv.s,
                     sv.Big + sv.s * n3, sv.sBig, sv.nk, ctx->stream, sv.kjac, d.N);
    PROF_END(PROF_APPLY, 0, (double)sv.njac * 3.0 * d.N * sv.s * (sizeof(C_t<R>) + 16.0));
    KCHK(hipGetLastError());
  }
  if (sv.npen > 0) {  // the pencil factors (plane-wave basis): forward and backward super-block solves
    Design& d = *sv.d;
    launch_pair<C_t<R>>((C_t<R>*)sv.Rp, n3, n3 * sv.s, sv.s, d.N, d.Np, sv.nk, -1, ctx->stream, sv.kpen);
    KCHK(potrs_batched<R>((const C_t<R>*)sv.A, (int)n3, n3, n3 * n3, sv.nk, (const C_t<R>*)sv.Dinv,
                          (n3 / 64) * 4096, (C_t<R>*)sv.Rp, n3, n3 * sv.s, (C_t<R>*)sv.Zp, n3, n3 * sv.s, sv.s,
                          ctx->stream, ctx->hk(), (const C_t<R>*)sv.SBinv, sv.kpen, sv.fmap, sv.npen));
    launch_pair<C_t<R>>((C_t<R>*)sv.Rp, n3, n3 * sv.s, sv.s, d.N, d.Np, sv.nk, 1, ctx->stream, sv.kpen);
    launch_widen<R>((const C_t<R>*)sv.Rp, n3 * sv.s, n3 * sv.s, sv.Big + sv.s * n3, sv.sBig, sv.nk, ctx->stream,
                    sv.kpen);
    KCHK(hipGetLastError());
  }
}

int choose_block(phx_ctx* ctx, int nb, int N) { return phx_host::choose_block(ctx->opt.block, nb, N); }

long per_k_bytes(const Design& d, int s, int prec, int precond) {
  return phx_host::per_k_bytes(d.n3, d.Np, s, prec, precond);
}

// Pencil preconditioner: A = K + sigma Omega assembled and Cholesky-factored for the
// k-points with which[k] != 0 (every k of the chunk at the start with precond 0; with
// precond 2, the k-points whose block-Jacobi iteration stalled), appended after the sv.nf
// factors built before; fmap_h (host, per k) receives each such k-point's factor index.
// Consecutive k-points of `which` within kshare_dist of a group's first k-point, and within
// kshare_rel of the shorter of the two wave vectors (at most kshare of them), share that
// k-point's factor; the shared solves need the super-block inverses.  The relative bound
// keeps Gamma, where K has the three rigid translations as null vectors and the factor is
// far from that of any other k, on a factor of its own.  cap: the number of factors the
// arrays hold (set by the first call of a solve).
template <typename R>
void build_factors(Solver& sv, const double* q, const std::vector<int>& which, std::vector<int>& fmap_h, int cap,
                   bool coarse) {
  phx_ctx* ctx = sv.ctx;
  Design& d = *sv.d;
  hipStream_t st = ctx->stream;
  const int nk = sv.nk;
  const long n3 = sv.n3;
  std::vector<int> lead;
  {
    std::vector<double> qc(3L * nk);
    std::vector<char> w(nk);
    for (int k = 0; k < nk; ++k) {
      w[k] = which[k] != 0;
      for (int c = 0; c < 3; ++c)
        qc[3 * k + c] = q[3 * k] * d.rec.t[0][c] + q[3 * k + 1] * d.rec.t[1][c] + q[3 * k + 2] * d.rec.t[2][c];
    }
    phx_host::share_groups(qc.data(), nk, w.data(), ctx->opt.sbinv ? ctx->opt.kshare : 1, ctx->opt.kshare_dist,
                           ctx->opt.kshare_rel, sv.nf, fmap_h.data(), lead);
  }
  const int nnew = (int)lead.size();
  if (nnew == 0) return;
  if (sv.nf == 0) sv.fcap = std::max(cap, nnew);
  if (sv.nf + nnew > sv.fcap) fail(ctx, PHX_EHIP, "internal: pencil factor capacity exceeded");
  if (!coarse) ctx->stats.factors += nnew;
  constexpr int WS = sizeof(R) == 4 ? 256 : 128;
  const long nsb = (n3 + WS - 1) / WS, f0 = sv.nf;
  sv.A = dbuf<C_t<R>>(ctx, "A", (long)sv.fcap * n3 * n3);
  sv.Dinv = dbuf<C_t<R>>(ctx, "Dinv", (long)sv.fcap * (n3 / 64) * 4096);
  C_t<R>* A = (C_t<R>*)sv.A + f0 * n3 * n3;
  C_t<R>* Dinv = (C_t<R>*)sv.Dinv + f0 * (n3 / 64) * 4096;
  // identity map unless factors are shared or only some k-points have one
  const bool ident = f0 == 0 && nnew == nk;
  if (!ident) {
    sv.fmap = dbuf<int>(ctx, "fmap", nk);
    HIPCHK(hipMemcpyAsync(sv.fmap, fmap_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
  }
  PROF_BEGIN(PROF_ASSEMBLE);
  const double* Kvf = sv.Kv;
  if (!ident) {  // wave vectors of the new factors' k-points
    double* kf = dbuf<double>(ctx, "Kvf", (long)sv.fcap * d.Np * 3);
    for (int i = 0; i < nnew; ++i)
      HIPCHK(hipMemcpyAsync(kf + (long)i * d.Np * 3, sv.Kv + (long)lead[i] * d.Np * 3, d.Np * 3 * sizeof(double),
                            hipMemcpyDeviceToDevice, st));
    Kvf = kf;
  }
  launch_assemble<R>(d.Dm, d.Bm, d.Os, Kvf, d.N, d.Np, nnew, d.c2, sv.sigma_d, A, n3 * n3, 0, st);
  // algorithmic bytes: the lower triangle of every A(k) written once, the three N x N operators read once
  PROF_END(PROF_ASSEMBLE, 0, (double)sizeof(C_t<R>) * nnew * (3.0 * d.N) * (3.0 * d.N + 1) / 2 + 48.0 * d.N * d.N);
  KCHK(hipGetLastError());
  KCHK(potrf_batched<R>(A, (int)n3, n3, n3 * n3, nnew, Dinv, (n3 / 64) * 4096, ctx->dflag, st, ctx->hk()));
  if (ctx->opt.sbinv) {
    sv.SBinv = dbuf<C_t<R>>(ctx, "SBinv", (long)sv.fcap * nsb * WS * WS);
    C_t<R>* sbw = dbuf<C_t<R>>(ctx, "SBwork", (long)sv.fcap * nsb * (WS * WS + WS * WS / 4));
    PROF_BEGIN(PROF_SBINV);
    KCHK(sb_inverse_batched<R>(A, (int)n3, n3, n3 * n3, nnew, Dinv, (n3 / 64) * 4096,
                               (C_t<R>*)sv.SBinv + f0 * nsb * WS * WS, sbw, st));
    PROF_END(PROF_SBINV, (double)nnew * 8.0 * n3 * WS * WS / 6.0, (double)nnew * sizeof(C_t<R>) * n3 * WS);
  } else if (!ident) {
    fail(ctx, PHX_EINVAL, "a partial or shared set of pencil factors needs option sbinv = 1");
  }
  sv.nf += nnew;
}

// init (may be NULL): nk blocks of s start vectors (n3 x s, k-stride n3 s) replacing
// the plane-wave unit vectors; tol_override > 0 replaces the precision's tolerance.
template <typename R>
void solve_chunk(phx_ctx* ctx, Design& d, const double* q, int nk, int nb, ChunkOut& out, Solver& sv,
                 const double2* init = nullptr, double tol_override = 0) {
  hipStream_t st = ctx->stream;
  const int prec = std::is_same<R, double>::value ? PHX_FP64 : PHX_MIXED;
  const int s = choose_block(ctx, nb, d.N), m = 3 * s;
  const long n3 = d.n3;
  sv.ctx = ctx; sv.d = &d; sv.nk = nk; sv.nb = nb; sv.s = s; sv.m = m; sv.prec = prec;
  sv.n3 = n3;
  sv.sBig = 3 * n3 * m;
  sv.Big = dbuf<double2>(ctx, "Big", (long)nk * sv.sBig);
  sv.Kv = dbuf<double>(ctx, "Kv", (long)nk * d.Np * 3);
  sv.sigma_d = dbuf<double>(ctx, "sigma", nk);
  sv.Y = dbuf<double2>(ctx, "Y", (long)nk * d.Np * 6 * s);
  sv.Tr = dbuf<double2>(ctx, "Tr", (long)nk * d.Np * s);
  sv.Zy = dbuf<double2>(ctx, "Zy", (long)nk * d.Np * 6 * s);
  sv.Zt = dbuf<double2>(ctx, "Zt", (long)nk * d.Np * s);
  sv.ksplit = ctx->opt.gram_split > 0 ? ctx->opt.gram_split
                                      : (int)std::max<long>(1, std::min<long>(16, n3 / 256));
  sv.G = dbuf<double2>(ctx, "G", (long)nk * m * m);
  sv.Gpart = dbuf<double2>(ctx, "Gpart", (long)sv.ksplit * nk * m * m);
  sv.C0 = dbuf<double2>(ctx, "C0", (long)nk * m * m);
  sv.Cr = dbuf<double2>(ctx, "Cr", (long)nk * m * s);
  sv.Cp = dbuf<double2>(ctx, "Cp", (long)nk * m * 2 * s);
  sv.G2 = dbuf<double2>(ctx, "G2", (long)nk * 2 * m * m);
  sv.G2part = dbuf<double2>(ctx, "G2part", (long)sv.ksplit * nk * 2 * m * m);
  sv.keep = dbuf<int>(ctx, "keep", (long)nk * m);
  sv.sweeps = dbuf<int>(ctx, "sweeps", nk);
  sv.kact = dbuf<int>(ctx, "kact", nk);
  sv.theta = dbuf<double>(ctx, "theta", (long)nk * s);
  sv.rn = dbuf<double>(ctx, "rn", (long)nk * s);
  sv.rnorm = dbuf<double>(ctx, "rnorm", (long)nk * s);
  sv.Rp = dbuf<C_t<R>>(ctx, "Rp", (long)nk * n3 * s);
  sv.Zp = dbuf<C_t<R>>(ctx, "Zp", (long)nk * n3 * s);
  double* qd = dbuf<double>(ctx, "q", 3L * nk);
  int* idx_d = dbuf<int>(ctx, "idx", (long)nk * s);

  // k-vectors, shift, initial plane-wave vectors
  HIPCHK(hipMemcpyAsync(qd, q, 3L * nk * sizeof(double), hipMemcpyHostToDevice, st));
  launch_kvec(qd, d.rec, d.M, d.N, d.Np, nk, sv.Kv, st);
  std::vector<double> sig(nk, d.sigma);
  HIPCHK(hipMemcpyAsync(sv.sigma_d, sig.data(), nk * sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<int> idx((size_t)nk * s);
  {
    const int L = 2 * d.M + 1;
    std::vector<int> ord(d.N);
    std::vector<double> k2(d.N);
    for (int k = 0; k < nk; ++k) {
      for (int p = 0; p < d.N; ++p) {
        const double n1 = p / (L * L) - d.M, n2 = (p / L) % L - d.M, n3_ = p % L - d.M;
        const double x[3] = {q[3 * k] + n1, q[3 * k + 1] + n2, q[3 * k + 2] + n3_};
        double kk = 0;
        for (int c = 0; c < 3; ++c) {
          const double kc = x[0] * d.rec.t[0][c] + x[1] * d.rec.t[1][c] + x[2] * d.rec.t[2][c];
          kk += kc * kc;
        }
        k2[p] = kk;
      }
      std::iota(ord.begin(), ord.end(), 0);
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return k2[a] < k2[b]; });
      for (int j = 0; j < s; ++j) idx[(size_t)k * s + j] = (j % 3) * d.Np + ord[j / 3];
    }
  }
  HIPCHK(hipMemcpyAsync(idx_d, idx.data(), idx.size() * sizeof(int), hipMemcpyHostToDevice, st));

  // The pencil preconditioner from the start (precond 0), or block Jacobi first (1, 2).
  HIPCHK(hipMemsetAsync(ctx->dflag, 0, sizeof(int), st));
  std::vector<int> fmap_h(nk, 0), pen_h(nk, ctx->opt.precond == 0 ? 1 : 0);
  sv.nf = sv.fcap = 0;
  sv.fmap = nullptr;
  sv.SBinv = nullptr;
  if (ctx->opt.precond == 0) build_factors<R>(sv, q, pen_h, fmap_h, nk, tol_override > 0);

  // Per-k activity: every k-point starts active; one whose wanted bands all meet the
  // tolerance is frozen (its basis, Ritz values and residual norms stay as they were)
  // and the remaining iterations skip it.  An active k-point is "far" until its own
  // residual falls below 1e-13/tol, then "near" (see the loop).  Every choice is made per
  // k-point, so a k-point's iterates do not depend on which other k-points share its chunk.
  std::vector<int> act_h(nk, 1), far_h(nk, 1), near_h(nk, 0), jac_h(nk), penm_h(nk);
  std::vector<char> near_k(nk, 0);
  sv.kfar = dbuf<int>(ctx, "kfar", nk);
  sv.knear = dbuf<int>(ctx, "knear", nk);
  sv.lact = dbuf<int>(ctx, "klist", 3L * nk);
  sv.lfar = sv.lact + nk;
  sv.lnear = sv.lact + 2 * nk;
  // the search directions of the next step that are not zero (their column is not soft
  // locked): a list of k * s + j and a mask per k * s + j, rebuilt every iteration
  int* wl_d = dbuf<int>(ctx, "wcols", 2L * nk * s);
  int* wm_d = wl_d + (long)nk * s;
  std::vector<int> wcols_h(2L * nk * s);
  // the lists of the active, far and near k-points, from the host masks
  std::vector<int> lists_h(3L * nk);
  auto upload_lists = [&](const std::vector<int>& a, const std::vector<int>& f, const std::vector<int>& n) {
    int na = 0, nf = 0, nn = 0;
    for (int k = 0; k < nk; ++k) {
      if (a[k]) lists_h[na++] = k;
      if (f[k]) lists_h[nk + nf++] = k;
      if (n[k]) lists_h[2 * nk + nn++] = k;
    }
    HIPCHK(hipMemcpyAsync(sv.lact, lists_h.data(), 3L * nk * sizeof(int), hipMemcpyHostToDevice, st));
  };
  sv.kjac = dbuf<int>(ctx, "kjac", nk);
  sv.kpen = dbuf<int>(ctx, "kpen", nk);
  for (int k = 0; k < nk; ++k) {
    jac_h[k] = !pen_h[k];
    penm_h[k] = pen_h[k];
  }
  HIPCHK(hipMemcpyAsync(sv.kact, act_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(sv.kfar, far_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(sv.knear, near_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(sv.kjac, jac_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(sv.kpen, penm_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
  upload_lists(act_h, far_h, near_h);
  sv.nact = sv.nfar = nk;
  sv.nnear = 0;
  sv.njac = ctx->opt.precond == 0 ? 0 : nk;
  sv.npen = nk - sv.njac;

  // Initial block: unit vectors of the smallest |K_p| (or the given start vectors); W = P = 0.
  launch_zero(sv.Big, (long)nk * sv.sBig, st);
  if (init) {
    HIPCHK(hipMemcpy2DAsync(sv.Big, sv.sBig * sizeof(double2), init, n3 * s * sizeof(double2), n3 * s * sizeof(double2),
                            nk, hipMemcpyDeviceToDevice, st));
  } else {
    launch_unit_columns(sv.Big, n3, sv.sBig, idx_d, s, nk, st, d.Np, d.N);
  }
  KCHK(hipGetLastError());
  apply_ops(sv, sv.Big, 0, s);

  const double tol = tol_override > 0 ? tol_override : ctx->opt.tol[prec];
  // the guard vectors (columns nb .. s-1) are not results: they may lock at a looser
  // threshold (option guard_lock; the coarse start keeps one threshold)
  const double gtol = tol_override > 0 ? tol : tol * ctx->opt.guard_lock;
  std::vector<double> rn_h((size_t)nk * s), rnorm_h((size_t)nk * s);
  std::vector<int> sw_h(nk);
  std::vector<char> kdone(nk, 0);
  std::vector<double> whist;  // per iteration and k: the largest residual of the wanted bands
  out.converged = false;
  int it = 0;
  for (it = 0; it <= ctx->opt.maxit; ++it) {
    const Sel all{sv.kact, sv.nact, sv.lact}, far{sv.kfar, sv.nfar, sv.lfar}, nearsel{sv.knear, sv.nnear, sv.lnear};
    // before the first step W and P are zero (the basis was cleared and only X written);
    // after it, the columns the last residual kernel locked are
    sv.zc = ctx->opt.zskip ? ZeroCols{sv.rn, tol, gtol, s, nb, it == 0 ? 1 : 0} : ZeroCols{nullptr, 0, 0, 0, 0, 0};
    // rr_fused 2: a k-point far from convergence takes both orthonormalisations in the small
    // space (one Gram product and one basis update per iteration); otherwise one explicit
    // Omega-CholQR of the basis first
    if (ctx->opt.rr_fused == 2) {
      if (sv.nnear > 0) cholqr(sv, nearsel);
    } else {
      cholqr(sv, all);
    }
    // The folded form multiplies the Gram matrix of K by the second orthonormalisation's
    // coefficients in the small space, which amplifies its rounding when the basis is
    // nearly dependent; near convergence (a k-point whose residual is below 1e-13/tol)
    // the second orthonormalisation is applied to the basis explicitly.
    if (ctx->opt.rr_fused) {
      if (sv.nfar > 0) rayleigh_ritz_fused(sv, far);
      if (sv.nnear > 0) {
        cholqr(sv, nearsel);
        rayleigh_ritz(sv, nearsel);
      }
    } else {
      cholqr(sv, all);
      rayleigh_ritz(sv, all);
    }
    // The images K X, Omega X (and those of the previous direction P) follow the basis
    // through the same coefficient updates.  Their rounding drift grows like the unit
    // roundoff over the size of P, which shrinks with the residual, so once a k-point's
    // residual is small enough for that drift to reach the tolerance its images are
    // recomputed from the vectors every iteration (with FP64 unit roundoff: residual below
    // 1e-13/tol, i.e. only the last iterations of an FP64-tolerance solve).
    if (sv.nnear > 0) {
      apply_ops(sv, sv.Big, 0, s, sv.knear, sv.nnear, sv.lnear);
      apply_ops(sv, sv.Big, 2 * s, s, sv.knear, sv.nnear, sv.lnear);
    }
    PROF_BEGIN(PROF_RESIDUAL);
    launch_residual<R>(sv.Big, n3, m, sv.sBig, sv.theta, s, nk, sv.sigma_d, tol, (C_t<R>*)sv.Rp, n3 * s,
                       sv.rn, sv.rnorm, st, sv.kact, nb, gtol);
    PROF_END(PROF_RESIDUAL, 0, 16.0 * 2 * 3.0 * d.N * s * sv.nact + (double)sizeof(C_t<R>) * 3.0 * d.N * s * sv.nact);
    KCHK(hipGetLastError());
    // residual norms, Jacobi sweep counts and (first iteration) the factorisation flag,
    // through pinned memory on this stream, then one host wait
    {
      const size_t nrn = rn_h.size() * sizeof(double), nsw = sw_h.size() * sizeof(int);
      char* hp = (char*)hbuf(ctx, nrn + nsw + sizeof(int));
      HIPCHK(hipMemcpyAsync(hp, sv.rn, nrn, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hp + nrn, sv.sweeps, nsw, hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hp + nrn + nsw, ctx->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
      wait_stream(ctx, st);
      memcpy(rn_h.data(), hp, nrn);
      memcpy(sw_h.data(), hp + nrn, nsw);
      int flag = 0;
      memcpy(&flag, hp + nrn + nsw, sizeof(int));
      if (flag) fail(ctx, PHX_ENOTPD, "pencil K + sigma Omega failed its Cholesky factorisation");
    }
    for (int v : sw_h) ctx->stats.rr_sweeps = std::max(ctx->stats.rr_sweeps, v);
    ctx->prof.flush();
    double worst = 0;
    for (int k = 0; k < nk; ++k) {
      double wk = 0;
      for (int j = 0; j < nb; ++j) wk = std::max(wk, rn_h[(size_t)k * s + j]);
      if (wk <= tol && !kdone[k]) {
        kdone[k] = 1;
        if (ctx->opt.kskip) act_h[k] = 0;
        if (!tol_override) {
          ctx->stats.k_conv_iters += it;
          ctx->stats.k_count += 1;
        }
      }
      if (!(wk == wk)) fail(ctx, PHX_EHIP, "eigensolver produced a non-finite residual");
      whist.push_back(wk);
      if (wk < 1e-13 / tol) near_k[k] = 1;
      worst = std::max(worst, wk);
    }
    if (ctx->trace) {
      std::vector<int> kh((size_t)nk * m);
      std::vector<double> th((size_t)nk * s);
      HIPCHK(hipMemcpy(kh.data(), sv.keep, kh.size() * sizeof(int), hipMemcpyDeviceToHost));
      HIPCHK(hipMemcpy(th.data(), sv.theta, th.size() * sizeof(double), hipMemcpyDeviceToHost));
      int kept = 0;
      for (int j = 0; j < m; ++j) kept += kh[j];
      double wall = 0;
      for (double v : rn_h) wall = std::max(wall, v);
      fprintf(stderr, "[phx] it %d worst(wanted) %.3e worst(all) %.3e kept(k0) %d theta(k0)", it, worst, wall, kept);
      for (int j = 0; j < std::min(s, 6); ++j) fprintf(stderr, " %.6g", th[j]);
      fprintf(stderr, " rn(k0)");
      for (int j = 0; j < std::min(s, 6); ++j) fprintf(stderr, " %.2e", rn_h[j]);
      fprintf(stderr, "\n");
    }
    if (worst <= tol) {
      out.converged = true;
      break;
    }
    if (it == ctx->opt.maxit) break;
    // precond 2: block Jacobi while it converges; a k-point still iterating whose residual
    // has not fallen tenfold over the last four iterations (or that reaches 30) gets its
    // own pencil factor (shared with k-points that stall in the same iteration, as
    // "kshare" allows) and is preconditioned by it from here on.  The decision is per
    // k-point, like every other decision of the iteration.
    if (ctx->opt.precond == 2) {
      std::vector<int> stall(nk, 0);
      int nst = 0;
      for (int k = 0; k < nk; ++k) {
        if (!act_h[k] || pen_h[k]) continue;
        const int w = ctx->opt.stall_its;
        stall[k] = it >= 30 || (it >= w && whist[(size_t)it * nk + k] > 0.1 * whist[(size_t)(it - w) * nk + k]);
        nst += stall[k];
      }
      if (nst > 0) {
        int cap = 0;  // the k-points that may still need a factor
        for (int k = 0; k < nk; ++k) cap += act_h[k] && !pen_h[k];
        build_factors<R>(sv, q, stall, fmap_h, cap, tol_override > 0);
        for (int k = 0; k < nk; ++k) pen_h[k] = pen_h[k] || stall[k];
        ctx->stats.precond_switches += nst;
      }
    }
    // masks for the next iteration
    {
      int na = 0, nf = 0, nn = 0, nj = 0, np = 0;
      bool chg = false;
      for (int k = 0; k < nk; ++k) {
        const int f = act_h[k] && !near_k[k], n = act_h[k] && near_k[k];
        const int j = act_h[k] && !pen_h[k], pm = act_h[k] && pen_h[k];
        chg = chg || f != far_h[k] || n != near_h[k] || j != jac_h[k] || pm != penm_h[k];
        far_h[k] = f;
        near_h[k] = n;
        jac_h[k] = j;
        penm_h[k] = pm;
        na += act_h[k];
        nf += f;
        nn += n;
        nj += j;
        np += pm;
      }
      if (chg) {
        HIPCHK(hipMemcpyAsync(sv.kact, act_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(sv.kfar, far_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(sv.knear, near_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(sv.kjac, jac_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(sv.kpen, penm_h.data(), nk * sizeof(int), hipMemcpyHostToDevice, st));
        upload_lists(act_h, far_h, near_h);
      }
      sv.nact = na;
      sv.nfar = nf;
      sv.nnear = nn;
      sv.njac = nj;
      sv.npen = np;
    }
    // The open columns of the active k-points, by the residual kernel's own test (a column
    // whose relative residual is below tol was soft locked there: its residual and the
    // images of its search direction are zero, and its direction will be zero).
    int nw = 0;
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < s; ++j) {
        const bool open = act_h[k] && !(rn_h[(size_t)k * s + j] < (j < nb ? tol : gtol));
        wcols_h[(size_t)nk * s + (size_t)k * s + j] = open;
        if (open) wcols_h[nw++] = k * s + j;
      }
    HIPCHK(hipMemcpyAsync(wl_d, wcols_h.data(), 2L * nk * s * sizeof(int), hipMemcpyHostToDevice, st));
    precondition<R>(sv);
    apply_ops(sv, sv.Big, s, s, nullptr, -1, nullptr, wl_d, nw, wm_d);
  }
  out.iters = it;
  out.theta.resize((size_t)nk * s);
  out.rnorm.resize((size_t)nk * s);
  out.rn = rn_h;
  HIPCHK(hipMemcpyAsync(out.theta.data(), sv.theta, out.theta.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(out.rnorm.data(), sv.rnorm, out.rnorm.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
}

// Adjoint of the converged chunk: d omega / d rho_e for bands sel (0-based) of
// every k of the chunk into out (device, (nk * nsel) x nvox).
void adjoint_chunk(Solver& sv, const std::vector<int>& sel, double* out) {
  phx_ctx* ctx = sv.ctx;
  Design& d = *sv.d;
  hipStream_t st = ctx->stream;
  const int nsel = (int)sel.size(), nk = sv.nk;
  const long n3 = sv.n3;
  int* sel_d = dbuf<int>(ctx, "sel", nsel);
  HIPCHK(hipMemcpyAsync(sel_d, sel.data(), nsel * sizeof(int), hipMemcpyHostToDevice, st));
  double2* Xs = dbuf<double2>(ctx, "Xsel", (long)nk * n3 * nsel);
  launch_gather_cols(sv.Big, n3, sv.sBig, sel_d, nsel, n3, nk, Xs, n3 * nsel, st);
  launch_pair<double2>(Xs, n3, n3 * nsel, nsel, d.N, d.Np, nk, -1, st);  // back to plane waves
  double* lam = dbuf<double>(ctx, "lam_sel", (long)nk * nsel);
  std::vector<double> th((size_t)nk * sv.s), lh((size_t)nk * nsel);
  HIPCHK(hipMemcpyAsync(th.data(), sv.theta, th.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int k = 0; k < nk; ++k)
    for (int j = 0; j < nsel; ++j) lh[(size_t)k * nsel + j] = th[(size_t)k * sv.s + sel[j]];
  HIPCHK(hipMemcpyAsync(lam, lh.data(), lh.size() * sizeof(double), hipMemcpyHostToDevice, st));
  double2* Y = dbuf<double2>(ctx, "Ysel", (long)nk * d.Np * 6 * nsel);
  double2* Tr = dbuf<double2>(ctx, "Trsel", (long)nk * d.Np * nsel);
  double2* Zy = dbuf<double2>(ctx, "Zysel", (long)nk * d.Np * 6 * nsel);
  double2* Zt = dbuf<double2>(ctx, "Ztsel", (long)nk * d.Np * nsel);
  launch_strain(Xs, n3, n3 * nsel, sv.Kv, d.Np, nsel, nk, Y, Tr, st);
  // the strain blocks of all k-points are contiguous: each compliance product is one wide
  // product (the operator read once, not once per k-point), always on 64 x 64 tiles, so a
  // k-point's result does not depend on how many k-points share the product
  gemm<double>(ctx, 0, 0, d.Np, 6 * nsel * nk, d.Np, 1, d.Bm, d.Np, 0, 1, Y, d.Np, 0, 1, Zy, d.Np, 0, ONE, ZERO, 1,
               nullptr, nullptr, 1, 0, 0, nullptr, 0, 2);
  gemm<double>(ctx, 0, 0, d.Np, nsel * nk, d.Np, 1, d.Dm, d.Np, 0, 1, Tr, d.Np, 0, 1, Zt, d.Np, 0, ONE, ZERO, 1,
               nullptr, nullptr, 1, 0, 0, nullptr, 0, 2);
  const long ncols = (long)nk * nsel;
  const int L = 2 * d.M + 1;
  double2* Fc = dbuf<double2>(ctx, "Fc", ncols * 9 * d.N);
  double2* H1 = dbuf<double2>(ctx, "H1", ncols * 9 * L * L * d.nv);
  double2* H2 = dbuf<double2>(ctx, "H2", ncols * 9 * L * (long)d.nv * d.nv);
  PROF_BEGIN(PROF_ADJOINT);
  launch_field_coef(Xs, n3, n3 * nsel, nsel, Zy, Zt, d.N, d.Np, nk, Fc, st);
  launch_synth(Fc, d.M, d.nv, ncols, H1, H2, st);
  launch_energy(H2, d.M, d.nv, (int)ncols, d.rho_d, d.mat, d.v, d.c2, lam, d.lscale, out, st);
  PROF_END(PROF_ADJOINT, 0, 8.0 * ncols * d.nvox + 16.0 * ncols * 9 * d.N);
  KCHK(hipGetLastError());
}

// Sensitivities of the requested bands sel (0-based) of every k of a converged chunk into
// out (device, (nk * nsel) x nvox), with the degenerate-cluster convention: the Ritz values
// theta (host, nk x s) are grouped into clusters of consecutive frequencies whose relative
// gap is below degen_tol, and a requested band inside a cluster of two or more receives the
// mean of the per-vector derivatives of all the cluster's members.  Eq. (15) holds for a
// simple eigenvalue only; inside a cluster any orthonormal basis of the eigenspace is as
// good as another and the per-vector values depend on it, while their sum (and so the mean)
// does not.  Returns the number of requested (k, band) entries that lie in a cluster.
long chunk_sensitivities(Solver& sv, const std::vector<double>& theta, const std::vector<int>& sel, double* out) {
  phx_ctx* ctx = sv.ctx;
  const int nk = sv.nk, s = sv.s, nsel = (int)sel.size();
  const phx_host::ClusterPlan pl = phx_host::cluster_plan(theta.data(), nk, s, sel.data(), nsel, ctx->opt.degen_tol);
  if (pl.ndeg == 0) {
    adjoint_chunk(sv, sel, out);
    return 0;
  }
  const int next = (int)pl.ext.size();
  const long nvox = sv.d->nvox;
  double* tmp = dbuf<double>(ctx, "sens_ext", (long)nk * next * nvox);
  adjoint_chunk(sv, pl.ext, tmp);
  const std::vector<double>& coef = pl.coef;
  double* cd = dbuf<double>(ctx, "sens_coef", (long)coef.size());
  HIPCHK(hipMemcpyAsync(cd, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  launch_combine_cols(tmp, next, cd, nsel, nk, nvox, out, ctx->stream);
  KCHK(hipGetLastError());
  // the host coefficients must outlive the copy
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return pl.ndeg;
}

// Runs the eigensolver over k-chunks; fills omega (+ err bounds) and, when sel is
// non-empty, the per-(k, band) sensitivities into sens_dev (device).
// dc (may be NULL): the same design at a lower plane-wave order; each chunk is then
// first solved there to a loose tolerance and its Ritz vectors start the full solve.
// A chunk whose workspaces do not fit (PHX_ENOMEM: a failed allocation, or the option
// mem_limit_gb) is retried with half as many k-points, down to one.
// Returns PHX_OK, PHX_ENOCONV, or PHX_WDEGEN when a requested band lies in a cluster.
int run_design(phx_ctx* ctx, Design& d, const double* q, int nk, int nb, int prec, double* omega, double* ebound,
               const std::vector<int>& sel, double* sens_dev, Design* dc = nullptr) {
  const int s = choose_block(ctx, nb, d.N);
  const long per = per_k_bytes(d, s, prec, ctx->opt.precond);
  int kc = phx_host::chunk_size(nk, ctx->opt.mem_gb, per);
  ctx->stats = Stats();
  ctx->stats.block = s;
  ctx->stats.kchunk = kc;
  // workspaces of earlier calls beyond the cap are given back first (they are grow-only)
  if (ctx->opt.mem_limit_gb > 0 && (double)ctx->mem_used > ctx->opt.mem_limit_gb * 1073741824.0)
    release_workspaces(ctx);
  bool conv = true;
  for (int k0 = 0; k0 < nk;) {
    const int nkc = std::min(kc, nk - k0);
    const Stats before = ctx->stats;
    ChunkOut co;
    Solver sv{};
    try {
      const double2* init = nullptr;
      if (dc) {
        ChunkOut cc;
        Solver svc{};
        if (prec == PHX_FP64) solve_chunk<double>(ctx, *dc, q + 3L * k0, nkc, nb, cc, svc, nullptr, ctx->opt.coarse_tol);
        else solve_chunk<float>(ctx, *dc, q + 3L * k0, nkc, nb, cc, svc, nullptr, ctx->opt.coarse_tol);
        ctx->stats.coarse_iters = std::max(ctx->stats.coarse_iters, cc.iters);
        double2* xi = dbuf<double2>(ctx, "Xinit", (long)nkc * d.n3 * s);
        launch_zero(xi, (long)nkc * d.n3 * s, ctx->stream);
        launch_prolong(svc.Big, dc->n3, svc.sBig, dc->M, dc->Np, xi, d.n3, d.n3 * s, d.M, d.Np, s, nkc, ctx->stream);
        KCHK(hipGetLastError());
        init = xi;
      }
      if (prec == PHX_FP64) solve_chunk<double>(ctx, d, q + 3L * k0, nkc, nb, co, sv, init);
      else solve_chunk<float>(ctx, d, q + 3L * k0, nkc, nb, co, sv, init);
      if (!sel.empty())
        ctx->stats.degen += chunk_sensitivities(sv, co.theta, sel, sens_dev + (long)k0 * sel.size() * d.nvox);
    } catch (const Fail& f) {
      if (f.code != PHX_ENOMEM || kc == 1) throw;
      const std::string why = ctx->err;
      release_workspaces(ctx);
      ctx->stats = before;
      kc = std::max(1, kc / 2);
      ctx->stats.kchunk = kc;
      ctx->stats.enomem_retries++;
      if (ctx->trace) fprintf(stderr, "[phx] %s: retrying with %d k-points per chunk\n", why.c_str(), kc);
      continue;
    }
    ctx->stats.chunks++;
    ctx->stats.iters = std::max(ctx->stats.iters, co.iters);
    conv = conv && co.converged;
    for (int k = 0; k < nkc; ++k)
      for (int j = 0; j < nb; ++j) {
        const double lam = co.theta[(size_t)k * s + j];
        const double om = sqrt(std::max(lam, 0.0) * d.lscale);
        if (omega) omega[(size_t)(k0 + k) * nb + j] = om;
        if (ebound) {
          const double bl = d.lscale * co.rnorm[(size_t)k * s + j] / sqrt(d.V * d.dens_min);
          ebound[(size_t)(k0 + k) * nb + j] = om > 0 ? std::min(bl / om, sqrt(bl)) : sqrt(bl);
        }
      }
    k0 += nkc;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->prof.flush();
  if (!conv) {
    ctx->err = "eigensolver reached maxit before every band met the tolerance";
    return PHX_ENOCONV;
  }
  if (ctx->stats.degen > 0) {
    ctx->err = std::to_string(ctx->stats.degen) +
               " requested (k, band) entries lie in degenerate clusters; their sensitivities are cluster means";
    return PHX_WDEGEN;
  }
  return PHX_OK;
}

// The same design at plane-wave order M-2, used to start the order-M eigensolver
// (enabled by the option "coarse" for M >= 4), or NULL.
Design* coarse_design(phx_ctx* ctx, const phx_cell& cell, const double* rho_host, const double* rho_dev, Design& dc) {
  if (!ctx->opt.coarse || cell.M < 4) return nullptr;
  phx_cell cc = cell;
  cc.M = std::max(1, cell.M - ctx->opt.coarse_drop);
  setup_design(ctx, cc, rho_host, rho_dev, dc, "c0:");
  return &dc;
}

// Status of several solves: the first error wins (caller's business), then PHX_ENOCONV,
// then the warning PHX_WDEGEN, then PHX_OK.
int worse_status(int a, int b) {
  auto rank = [](int r) { return r == PHX_ENOCONV ? 2 : (r == PHX_WDEGEN ? 1 : 0); };
  return rank(b) > rank(a) ? b : a;
}

int guard(phx_ctx* ctx, const std::function<int()>& f) {
  if (!ctx) return PHX_EINVAL;
  ctx->err.clear();
  try {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) {
      ctx->err = std::string("hipSetDevice: ") + hipGetErrorString(e);
      return PHX_EHIP;
    }
    return f();
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::exception& ex) {
    ctx->err = ex.what();
    return PHX_EHIP;
  }
}

void check_bands(phx_ctx* ctx, const phx_cell* cell, int nb, int nsens, const int* band_no) {
  if (const char* e = phx_host::check_bands(cell, nb, nsens, band_no, ctx->opt.block)) fail(ctx, PHX_EINVAL, e);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int phx_create(phx_ctx** out, int hip_device) {
  if (!out) return PHX_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return PHX_EHIP;
  if (hip_device < 0 || hip_device >= n) return PHX_EINVAL;
  phx_ctx* c = new phx_ctx();
  c->device = hip_device;
  const char* tr = getenv("PHX_TRACE");
  c->trace = tr && tr[0] && tr[0] != '0';
  if (hipSetDevice(hip_device) != hipSuccess || scratch_setup(hip_device) != PHX_OK ||
      hipStreamCreate(&c->stream) != hipSuccess || hipMalloc(&c->dflag, sizeof(int)) != hipSuccess ||
      hipEventCreateWithFlags(&c->wait_ev, hipEventBlockingSync | hipEventDisableTiming) != hipSuccess) {
    if (c->dflag) (void)hipFree(c->dflag);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return PHX_EHIP;
  }
  c->prof.st = c->stream;
  *out = c;
  return PHX_OK;
}

int phx_destroy(phx_ctx* ctx) {
  if (!ctx) return PHX_EINVAL;
  for (phx_ctx* w : ctx->workers) phx_destroy(w);
  ctx->workers.clear();
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (ctx->dflag) (void)hipFree(ctx->dflag);
  if (ctx->hpin) (void)hipHostFree(ctx->hpin);
  if (ctx->wait_ev) (void)hipEventDestroy(ctx->wait_ev);
  if (ctx->stream && ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return PHX_OK;
}

const char* phx_last_error(const phx_ctx* ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

int phx_set_option(phx_ctx* ctx, const char* key, double v) {
  if (!ctx || !key) return PHX_EINVAL;
  std::string k(key);
  auto bad = [&]() {
    ctx->err = "bad value for option " + k;
    return PHX_EINVAL;
  };
  if (k == "tol_fp64") { if (!(v > 0 && v < 1)) return bad(); ctx->opt.tol[0] = v; }
  else if (k == "tol_mixed") { if (!(v > 0 && v < 1)) return bad(); ctx->opt.tol[1] = v; }
  else if (k == "maxit") { if (!(v >= 1 && v <= 10000)) return bad(); ctx->opt.maxit = (int)v; }
  else if (k == "block") { if (!(v == 0 || (v >= 2 && v <= 21))) return bad(); ctx->opt.block = (int)v; }
  else if (k == "shift") { if (!(v > 0 && v < 1e6)) return bad(); ctx->opt.shift = v; }
  else if (k == "drop") { if (!(v > 0 && v < 1e-2)) return bad(); ctx->opt.drop = v; }
  else if (k == "mem_gb") { if (!(v > 0)) return bad(); ctx->opt.mem_gb = v; }
  else if (k == "coarse") { if (!(v == 0 || v == 1)) return bad(); ctx->opt.coarse = (int)v; }
  else if (k == "coarse_tol") { if (!(v > 0 && v < 1)) return bad(); ctx->opt.coarse_tol = v; }
  else if (k == "coarse_drop") { if (!(v >= 1 && v <= 3 && v == (int)v)) return bad(); ctx->opt.coarse_drop = (int)v; }
  else if (k == "streams") { if (!(v >= 1 && v <= 16)) return bad(); ctx->opt.streams = (int)v; }
  else if (k == "rr_fused") { if (!(v == 0 || v == 1 || v == 2)) return bad(); ctx->opt.rr_fused = (int)v; }
  else if (k == "small_eig") { if (!(v == 0 || v == 1)) return bad(); ctx->opt.small_eig = (int)v; }
  else if (k == "sbinv") { if (!(v == 0 || v == 1)) return bad(); ctx->opt.sbinv = (int)v; }
  else if (k == "kskip") { if (!(v == 0 || v == 1)) return bad(); ctx->opt.kskip = (int)v; }
  else if (k == "kshare") { if (!(v >= 1 && v <= 8 && v == (int)v)) return bad(); ctx->opt.kshare = (int)v; }
  else if (k == "kshare_dist") { if (!(v >= 0 && v <= 1)) return bad(); ctx->opt.kshare_dist = v; }
  else if (k == "kshare_rel") { if (!(v >= 0 && v <= 1)) return bad(); ctx->opt.kshare_rel = v; }
  else if (k == "kstreams") { if (!(v >= 1 && v <= 16 && v == (int)v)) return bad(); ctx->opt.kstreams = (int)v; }
  else if (k == "gram_split") { if (!(v >= 0 && v <= 16 && v == (int)v)) return bad(); ctx->opt.gram_split = (int)v; }
  else if (k == "spin_wait") { if (!(v == 0 || v == 1)) return bad(); ctx->opt.spin_wait = (int)v; }
  else if (k == "omega_conv") { if (!(v == 0 || v == 1)) return bad(); ctx->opt.omega_conv = (int)v; }
  else if (k == "guard_lock") { if (!(v >= 1 && v <= 1e4)) return bad(); ctx->opt.guard_lock = v; }
  else if (k == "zskip") { if (!(v == 0 || v == 1)) return bad(); ctx->opt.zskip = (int)v; }
  else if (k == "degen_tol") { if (!(v >= 0 && v < 1e-2)) return bad(); ctx->opt.degen_tol = v; }
  else if (k == "mem_limit_gb") { if (!(v >= 0 && v < 1e6)) return bad(); ctx->opt.mem_limit_gb = v; }
  else if (k == "precond") { if (!(v == 0 || v == 1 || v == 2)) return bad(); ctx->opt.precond = (int)v; }
  else if (k == "stall_its") { if (!(v >= 2 && v <= 30 && v == (int)v)) return bad(); ctx->opt.stall_its = (int)v; }
  else if (k == "profile") {
    if (!(v == 0 || v == 1 || v == 2)) return bad();
    ctx->prof.on = v != 0;
    ctx->prof.stages = v != 2;
  }
  else if (k == "profile_reset") { ctx->prof.reset(); }
  else { ctx->err = "unknown option " + k; return PHX_EINVAL; }
  return PHX_OK;
}

int phx_get_stat(const phx_ctx* ctx, const char* key, double* value) {
  if (!ctx || !key || !value) return PHX_EINVAL;
  std::string k(key);
  if (k == "iters") *value = ctx->stats.iters;
  else if (k == "chunks") *value = ctx->stats.chunks;
  else if (k == "block") *value = ctx->stats.block;
  else if (k == "kchunk") *value = ctx->stats.kchunk;
  else if (k == "rr_sweeps") *value = ctx->stats.rr_sweeps;
  else if (k == "coarse_iters") *value = ctx->stats.coarse_iters;
  else if (k == "factors") *value = (double)ctx->stats.factors;
  else if (k == "iters_mean_k") *value = ctx->stats.k_count ? (double)ctx->stats.k_conv_iters / ctx->stats.k_count : 0;
  else if (k == "degen") *value = (double)ctx->stats.degen;
  else if (k == "enomem_retries") *value = ctx->stats.enomem_retries;
  else if (k == "precond_switches") *value = ctx->stats.precond_switches;
  else if (k == "mem_bytes") *value = (double)ctx->mem_used;
  else if (k.rfind("prof.", 0) == 0) {
    const size_t dot = k.rfind('.');
    const std::string cls = k.substr(5, dot - 5), f = k.substr(dot + 1);
    int c = -1;
    for (int i = 0; i < PROF_NCLASS; ++i)
      if (cls == PROF_NAMES[i]) c = i;
    if (c < 0) return PHX_EINVAL;
    const ProfAcc& a = ctx->prof.acc[c];
    if (f == "ms") *value = a.ms;
    else if (f == "flops") *value = a.flops;
    else if (f == "bytes") *value = a.bytes;
    else if (f == "count") *value = (double)a.count;
    else return PHX_EINVAL;
  }
  else return PHX_EINVAL;
  return PHX_OK;
}

int phx_fourier(phx_ctx* ctx, const phx_cell* cell, const double* rho, double* out) {
  return guard(ctx, [&]() {
    check_cell(ctx, cell);
    if (!out) fail(ctx, PHX_EINVAL, "out is NULL");
    const long nvox = (long)cell->nv * cell->nv * cell->nv;
    check_rho(ctx, rho, nvox);
    Design d;
    setup_geometry(*cell, d);
    double* rd = dbuf<double>(ctx, "rho", nvox);
    HIPCHK(hipMemcpyAsync(rd, rho, nvox * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    const int L2 = 4 * d.M + 1;
    const long nt = (long)L2 * L2 * L2;
    double* F = dbuf<double>(ctx, "F", 3 * nvox);
    double2* G1 = dbuf<double2>(ctx, "G1", 3L * d.nv * d.nv * L2);
    double2* G2 = dbuf<double2>(ctx, "G2", 3L * d.nv * L2 * L2);
    double2* T = dbuf<double2>(ctx, "tab", 3 * nt);
    launch_fields(rd, (int)nvox, d.mat, F, ctx->stream);
    launch_dft(F, d.nv, d.M, d.v, G1, G2, T, ctx->stream);
    KCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, T, 3 * nt * sizeof(double2), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double a = cell->a;
    const double sc[3] = {a * a * a * cell->phase0.density, a * a * a / cell->phase0.youngs,
                          a * a * a / cell->phase0.youngs};
    for (int f = 0; f < 3; ++f)
      for (long i = 0; i < 2 * nt; ++i) out[f * 2 * nt + i] *= sc[f];
    return PHX_OK;
  });
}

int phx_schur(phx_ctx* ctx, const phx_cell* cell, const double* rho, const double* q, double* out) {
  return guard(ctx, [&]() {
    check_cell(ctx, cell);
    if (!out) fail(ctx, PHX_EINVAL, "out is NULL");
    const long nvox = (long)cell->nv * cell->nv * cell->nv;
    check_rho(ctx, rho, nvox);
    check_q(ctx, q, 1);
    Design d;
    setup_design(ctx, *cell, rho, nullptr, d, "d0:");
    hipStream_t st = ctx->stream;
    double* qd = dbuf<double>(ctx, "q", 3);
    double* Kv = dbuf<double>(ctx, "Kv", (long)d.Np * 3);
    double* sg = dbuf<double>(ctx, "sigma", 1);
    const long n3 = d.n3;
    double2* A = dbuf<double2>(ctx, "A", n3 * n3);
    HIPCHK(hipMemcpyAsync(qd, q, 3 * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(sg, 0, sizeof(double), st));
    launch_kvec(qd, d.rec, d.M, d.N, d.Np, 1, Kv, st);
    launch_assemble<double>(d.Dm, d.Bm, d.Os, Kv, d.N, d.Np, 1, d.c2, sg, A, n3 * n3, 1, st);
    KCHK(hipGetLastError());
    std::vector<double2> h(n3 * n3);
    HIPCHK(hipMemcpyAsync(h.data(), A, h.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const long n = 3L * d.N;
    const double sc = cell->a * cell->phase0.youngs;
    for (int cj = 0; cj < 3; ++cj)
      for (int qq = 0; qq < d.N; ++qq)
        for (int ci = 0; ci < 3; ++ci)
          for (int p = 0; p < d.N; ++p) {
            const double2 v = h[(ci * d.Np + p) + (long)(cj * d.Np + qq) * n3];
            const long o = (3L * p + ci) + (3L * qq + cj) * n;
            out[2 * o] = v.x * sc;
            out[2 * o + 1] = v.y * sc;
          }
    return PHX_OK;
  });
}

static int bands_impl(phx_ctx* ctx, const phx_cell* cell, const double* rho, int nk, const double* q, int nbands,
                      phx_precision prec, int nsens, const int* band_no, double* omega, double* ebound,
                      double* domega, const double* weight, double* grad) {
  check_cell(ctx, cell);
  const long nvox = (long)cell->nv * cell->nv * cell->nv;
  check_rho(ctx, rho, nvox);
  check_q(ctx, q, nk);
  check_bands(ctx, cell, nbands, nsens, band_no);
  if (prec != PHX_FP64 && prec != PHX_MIXED) fail(ctx, PHX_EINVAL, "unknown precision");
  Design d;
  setup_design(ctx, *cell, rho, nullptr, d, "d0:");
  std::vector<int> sel;
  for (int j = 0; j < nsens; ++j) sel.push_back(band_no[j] - 1);
  double* sens = nullptr;
  if (nsens > 0) sens = dbuf<double>(ctx, "sens", (long)nk * nsens * nvox);
  std::vector<double> om_tmp;
  if (!omega) {
    om_tmp.resize((size_t)nk * nbands);
    omega = om_tmp.data();
  }
  Design dcs;
  Design* dc = coarse_design(ctx, *cell, rho, nullptr, dcs);
  int rc = run_design(ctx, d, q, nk, nbands, prec, omega, ebound, sel, sens, dc);
  hipStream_t st = ctx->stream;
  if (nsens > 0 && domega) {
    HIPCHK(hipMemcpyAsync(domega, sens, (long)nk * nsens * nvox * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (nsens > 0 && grad) {
    double* w = dbuf<double>(ctx, "wgt", (long)nk * nsens);
    double* g = dbuf<double>(ctx, "grad", nvox);
    HIPCHK(hipMemcpyAsync(w, weight, (long)nk * nsens * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(g, 0, nvox * sizeof(double), st));
    launch_weighted_sum(sens, w, nk * nsens, nvox, g, st);
    KCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(grad, g, nvox * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return rc;
}

int phx_bands(phx_ctx* ctx, const phx_cell* cell, const double* rho, int nk, const double* q, int nbands,
              phx_precision prec, double* omega, double* err_bound) {
  return guard(ctx, [&]() {
    if (!omega) fail(ctx, PHX_EINVAL, "omega is NULL");
    return bands_impl(ctx, cell, rho, nk, q, nbands, prec, 0, nullptr, omega, err_bound, nullptr, nullptr, nullptr);
  });
}

int phx_sens(phx_ctx* ctx, const phx_cell* cell, const double* rho, int nk, const double* q, int nbands,
             phx_precision prec, int nsens, const int* band_no, double* omega, double* domega_drho) {
  return guard(ctx, [&]() {
    if (!omega || !domega_drho) fail(ctx, PHX_EINVAL, "omega or domega_drho is NULL");
    if (nsens < 1) fail(ctx, PHX_EINVAL, "nsens must be at least 1");
    return bands_impl(ctx, cell, rho, nk, q, nbands, prec, nsens, band_no, omega, nullptr, domega_drho, nullptr,
                      nullptr);
  });
}

int phx_adjoint(phx_ctx* ctx, const phx_cell* cell, const double* rho, int nk, const double* q, int nbands,
                phx_precision prec, int nsens, const int* band_no, const double* weight, double* omega,
                double* grad) {
  return guard(ctx, [&]() {
    if (!weight || !grad) fail(ctx, PHX_EINVAL, "weight or grad is NULL");
    if (nsens < 1) fail(ctx, PHX_EINVAL, "nsens must be at least 1");
    for (long i = 0; i < (long)nk * nsens; ++i)
      if (!isfinite(weight[i])) fail(ctx, PHX_EINVAL, "weights must be finite");
    return bands_impl(ctx, cell, rho, nk, q, nbands, prec, nsens, band_no, omega, nullptr, nullptr, weight, grad);
  });
}

int phx_bands_batch(phx_ctx* ctx, int ndesign, const phx_cell* cells, const double* const* rho, int nk,
                    const double* q, int nbands, phx_precision prec, int nsens, const int* band_no,
                    double* const* omega, double* const* domega) {
  return guard(ctx, [&]() {
    if (ndesign < 1 || !cells || !rho || !omega) fail(ctx, PHX_EINVAL, "ndesign, cells, rho and omega are required");
    int worst = PHX_OK;
    std::string msg, wmsg;
    for (int i = 0; i < ndesign; ++i) {
      if (!omega[i]) fail(ctx, PHX_EINVAL, "omega[d] is NULL");
      const int rc = bands_impl(ctx, &cells[i], rho[i], nk, q, nbands, prec, (domega && domega[i]) ? nsens : 0,
                                band_no, omega[i], nullptr, domega ? domega[i] : nullptr, nullptr, nullptr);
      if (rc != PHX_OK) msg = "design " + std::to_string(i) + ": " + ctx->err;
      if (worse_status(worst, rc) != worst) {
        worst = rc;
        wmsg = msg;
      }
    }
    ctx->err = wmsg;
    return worst;
  });
}

// Device-pointer path shared by the *_dev calls: rho on the device, q on the host,
// omega / domega / grad on the device (each may be NULL when not wanted).
static int dev_impl(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host,
                    int nbands, phx_precision prec, int nsens, const int* band_no, double* omega_dev,
                    double* domega_dev, const double* weight_dev, double* grad_dev, void* stream) {
  check_cell(ctx, cell);
  if (!rho_dev) fail(ctx, PHX_EINVAL, "rho_dev is NULL");
  check_q(ctx, q_host, nk);
  check_bands(ctx, cell, nbands, nsens, band_no);
  if (prec != PHX_FP64 && prec != PHX_MIXED) fail(ctx, PHX_EINVAL, "unknown precision");
  if (stream) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  const long nvox = (long)cell->nv * cell->nv * cell->nv;
  hipStream_t st = ctx->stream;
  std::vector<double> rh(nvox);
  HIPCHK(hipMemcpyAsync(rh.data(), rho_dev, nvox * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  check_rho(ctx, rh.data(), nvox);
  Design d;
  setup_design(ctx, *cell, rh.data(), rho_dev, d, "d0:");
  std::vector<int> sel;
  for (int j = 0; j < nsens; ++j) sel.push_back(band_no[j] - 1);
  double* sens = domega_dev;
  if (nsens > 0 && !sens) sens = dbuf<double>(ctx, "sens", (long)nk * nsens * nvox);
  std::vector<double> om((size_t)nk * nbands);
  Design dcs;
  Design* dc = coarse_design(ctx, *cell, rh.data(), rho_dev, dcs);
  const int rc = run_design(ctx, d, q_host, nk, nbands, prec, om.data(), nullptr, sel, sens, dc);
  if (omega_dev)
    HIPCHK(hipMemcpyAsync(omega_dev, om.data(), om.size() * sizeof(double), hipMemcpyHostToDevice, st));
  if (grad_dev) {
    HIPCHK(hipMemsetAsync(grad_dev, 0, nvox * sizeof(double), st));
    launch_weighted_sum(sens, weight_dev, nk * nsens, nvox, grad_dev, st);
    KCHK(hipGetLastError());
  }
  HIPCHK(hipStreamSynchronize(st));
  return rc;
}

// Worker contexts (own stream and workspaces) for concurrent solves, with the caller's
// options and profiling settings.
static void prepare_workers(phx_ctx* ctx, int nw) {
  while ((int)ctx->workers.size() < nw) {
    phx_ctx* w = nullptr;
    if (phx_create(&w, ctx->device) != PHX_OK) fail(ctx, PHX_EHIP, "could not create a worker stream");
    ctx->workers.push_back(w);
  }
  for (int i = 0; i < nw; ++i) {
    ctx->workers[i]->opt = ctx->opt;
    ctx->workers[i]->prof.on = ctx->prof.on;
    ctx->workers[i]->prof.stages = ctx->prof.stages;
    ctx->workers[i]->trace = ctx->trace;
  }
}

// The workers' timers and statistics into the caller's.
static void merge_workers(phx_ctx* ctx, int nw) {
  ctx->stats = Stats();
  for (int i = 0; i < nw; ++i) {
    phx_ctx* w = ctx->workers[i];
    for (int c = 0; c < PROF_NCLASS; ++c) {
      ctx->prof.acc[c].ms += w->prof.acc[c].ms;
      ctx->prof.acc[c].flops += w->prof.acc[c].flops;
      ctx->prof.acc[c].bytes += w->prof.acc[c].bytes;
      ctx->prof.acc[c].count += w->prof.acc[c].count;
    }
    w->prof.reset();
    merge_stats(ctx->stats, w->stats);
  }
}

// One design's k-points in ctx->opt.kstreams consecutive ranges, solved concurrently on
// worker streams (a single design leaves most of the GPU idle on one stream).  Each range
// writes its own rows of omega and of the sensitivities; for the weighted adjoint each
// range's gradient goes to a slice of a scratch array, summed into grad_dev afterwards.
static int dev_entry(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host,
                     int nbands, phx_precision prec, int nsens, const int* band_no, double* omega_dev,
                     double* domega_dev, const double* weight_dev, double* grad_dev, void* stream) {
  const int np = std::min(ctx->opt.kstreams, nk);
  if (np <= 1)
    return dev_impl(ctx, cell, rho_dev, nk, q_host, nbands, prec, nsens, band_no, omega_dev, domega_dev, weight_dev,
                    grad_dev, stream);
  check_cell(ctx, cell);
  check_q(ctx, q_host, nk);
  if (stream) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  const long nvox = (long)cell->nv * cell->nv * cell->nv;
  double* parts = grad_dev ? dbuf<double>(ctx, "gparts", (long)np * nvox) : nullptr;
  prepare_workers(ctx, np);
  std::vector<int> rcs(np, PHX_OK);
  std::vector<std::string> errs(np);
  std::vector<std::thread> th;
  for (int p = 0; p < np; ++p)
    th.emplace_back([&, p]() {
      phx_ctx* w = ctx->workers[p];
      const int k0 = (int)((long)nk * p / np), k1 = (int)((long)nk * (p + 1) / np);
      rcs[p] = guard(w, [&]() {
        return dev_impl(w, cell, rho_dev, k1 - k0, q_host + 3L * k0, nbands, prec, nsens, band_no,
                        omega_dev ? omega_dev + (long)k0 * nbands : nullptr,
                        domega_dev ? domega_dev + (long)k0 * nsens * nvox : nullptr,
                        weight_dev ? weight_dev + (long)k0 * nsens : nullptr,
                        parts ? parts + (long)p * nvox : nullptr, nullptr);
      });
      if (rcs[p] != PHX_OK) errs[p] = w->err;
    });
  for (auto& t : th) t.join();
  merge_workers(ctx, np);
  int worst = PHX_OK;
  for (int p = 0; p < np; ++p) {
    if (rcs[p] < 0 && rcs[p] != PHX_ENOCONV) {
      ctx->err = "k range " + std::to_string(p) + ": " + errs[p];
      return rcs[p];
    }
    if (worse_status(worst, rcs[p]) != worst) {
      worst = rcs[p];
      ctx->err = "k range " + std::to_string(p) + ": " + errs[p];
    }
  }
  if (grad_dev) {  // the workers' streams are done (each synchronised before its thread ended)
    std::vector<double> ones(np, 1.0);
    double* od = dbuf<double>(ctx, "gones", np);
    HIPCHK(hipMemcpyAsync(od, ones.data(), np * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemsetAsync(grad_dev, 0, nvox * sizeof(double), ctx->stream));
    launch_weighted_sum(parts, od, np, nvox, grad_dev, ctx->stream);
    KCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  return worst;
}

int phx_bands_dev(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host,
                  int nbands, phx_precision prec, double* omega_dev, void* stream) {
  return guard(ctx, [&]() {
    if (!omega_dev) fail(ctx, PHX_EINVAL, "omega_dev is NULL");
    return dev_entry(ctx, cell, rho_dev, nk, q_host, nbands, prec, 0, nullptr, omega_dev, nullptr, nullptr, nullptr,
                     stream);
  });
}

int phx_sens_dev(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host, int nbands,
                 phx_precision prec, int nsens, const int* band_no, double* omega_dev, double* domega_dev,
                 void* stream) {
  return guard(ctx, [&]() {
    if (!omega_dev) fail(ctx, PHX_EINVAL, "omega_dev is NULL");
    if (nsens > 0 && !domega_dev) fail(ctx, PHX_EINVAL, "domega_dev is NULL");
    return dev_entry(ctx, cell, rho_dev, nk, q_host, nbands, prec, nsens, band_no, omega_dev, domega_dev, nullptr,
                     nullptr, stream);
  });
}

int phx_adjoint_dev(phx_ctx* ctx, const phx_cell* cell, const double* rho_dev, int nk, const double* q_host,
                    int nbands, phx_precision prec, int nsens, const int* band_no, const double* weight_dev,
                    double* omega_dev, double* grad_dev, void* stream) {
  return guard(ctx, [&]() {
    if (!weight_dev || !grad_dev) fail(ctx, PHX_EINVAL, "weight_dev or grad_dev is NULL");
    if (nsens < 1) fail(ctx, PHX_EINVAL, "nsens must be at least 1");
    return dev_entry(ctx, cell, rho_dev, nk, q_host, nbands, prec, nsens, band_no, omega_dev, nullptr, weight_dev,
                     grad_dev, stream);
  });
}

int phx_sens_batch_dev(phx_ctx* ctx, int ndesign, const phx_cell* cells, const double* const* rho_dev, int nk,
                       const double* q_host, int nbands, phx_precision prec, int nsens, const int* band_no,
                       double* const* omega_dev, double* const* domega_dev, void* stream) {
  return guard(ctx, [&]() {
    if (ndesign < 1 || !cells || !rho_dev || !omega_dev) fail(ctx, PHX_EINVAL, "ndesign, cells, rho_dev and omega_dev are required");
    if (nsens > 0 && !domega_dev) fail(ctx, PHX_EINVAL, "domega_dev is NULL");
    check_q(ctx, q_host, nk);
    for (int d = 0; d < ndesign; ++d) {
      check_cell(ctx, &cells[d]);
      check_bands(ctx, &cells[d], nbands, nsens, band_no);
      if (!rho_dev[d] || !omega_dev[d] || (nsens > 0 && !domega_dev[d]))
        fail(ctx, PHX_EINVAL, "a per-design pointer is NULL");
    }
    if (prec != PHX_FP64 && prec != PHX_MIXED) fail(ctx, PHX_EINVAL, "unknown precision");
    if (stream) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int nw = std::min(ctx->opt.streams, ndesign);
    prepare_workers(ctx, nw);
    // most expensive designs first: the per-k cost grows like (3N)^3
    std::vector<int> order(ndesign);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cells[a].M > cells[b].M; });
    std::atomic<int> next(0);
    std::vector<int> rcs(ndesign, PHX_OK);
    std::vector<std::string> errs(ndesign);
    auto work = [&](phx_ctx* w) {
      Stats total;  // every design this worker solves (each solve resets w->stats)
      for (;;) {
        const int i = next.fetch_add(1);
        if (i >= ndesign) break;
        const int d = order[i];
        rcs[d] = guard(w, [&]() {
          return dev_impl(w, &cells[d], rho_dev[d], nk, q_host, nbands, prec, nsens, band_no, omega_dev[d],
                          nsens > 0 ? domega_dev[d] : nullptr, nullptr, nullptr, nullptr);
        });
        if (rcs[d] != PHX_OK) errs[d] = w->err;
        merge_stats(total, w->stats);
      }
      w->stats = total;
    };
    if (nw == 1) {
      work(ctx->workers[0]);
    } else {
      std::vector<std::thread> th;
      for (int i = 0; i < nw; ++i) th.emplace_back(work, ctx->workers[i]);
      for (auto& t : th) t.join();
    }
    merge_workers(ctx, nw);
    int worst = PHX_OK;
    for (int d = 0; d < ndesign; ++d) {
      if (rcs[d] < 0 && rcs[d] != PHX_ENOCONV) {
        ctx->err = "design " + std::to_string(d) + ": " + errs[d];
        return rcs[d];
      }
      if (worse_status(worst, rcs[d]) != worst) {
        worst = rcs[d];
        ctx->err = "design " + std::to_string(d) + ": " + errs[d];
      }
    }
    return worst;
  });
}

int phx_zgemm(phx_ctx* ctx, phx_precision prec, char opa, char opb, int m, int n, int k, const double* alpha,
              const double* A, long lda, long strideA, const double* B, long ldb, long strideB, const double* beta,
              double* C, long ldc, long strideC, int batch) {
  return guard(ctx, [&]() {
    if (m < 0 || n < 0 || k < 0 || batch < 1 || !alpha || !beta || !A || !B || !C)
      fail(ctx, PHX_EINVAL, "bad zgemm arguments");
    const int oa = (opa == 'C' || opa == 'c') ? 1 : 0, ob = (opb == 'C' || opb == 'c') ? 1 : 0;
    if ((opa != 'N' && opa != 'n' && !oa) || (opb != 'N' && opb != 'n' && !ob)) fail(ctx, PHX_EINVAL, "op must be N or C");
    const long ra = oa ? k : m, ca = oa ? m : k, rb = ob ? n : k, cb = ob ? k : n;
    if (lda < std::max<long>(1, ra) || ldb < std::max<long>(1, rb) || ldc < std::max<long>(1, m))
      fail(ctx, PHX_EINVAL, "leading dimension too small");
    const long na = strideA * (batch - 1) + lda * (ca - 1) + ra;
    const long nbb = strideB * (batch - 1) + ldb * (cb - 1) + rb;
    const long nc = strideC * (batch - 1) + ldc * (n - 1) + m;
    hipStream_t st = ctx->stream;
    auto run = [&](auto tag) {
      typedef decltype(tag) R;
      typedef C_t<R> Cx;
      std::vector<Cx> ha(na), hb(nbb), hc(nc);
      for (long i = 0; i < na; ++i) ha[i] = mk<R>((R)A[2 * i], (R)A[2 * i + 1]);
      for (long i = 0; i < nbb; ++i) hb[i] = mk<R>((R)B[2 * i], (R)B[2 * i + 1]);
      for (long i = 0; i < nc; ++i) hc[i] = mk<R>((R)C[2 * i], (R)C[2 * i + 1]);
      Cx* da = dbuf<Cx>(ctx, "tA", na);
      Cx* db = dbuf<Cx>(ctx, "tB", nbb);
      Cx* dc = dbuf<Cx>(ctx, "tC", nc);
      HIPCHK(hipMemcpyAsync(da, ha.data(), na * sizeof(Cx), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(db, hb.data(), nbb * sizeof(Cx), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(dc, hc.data(), nc * sizeof(Cx), hipMemcpyHostToDevice, st));
      gemm<R>(ctx, oa, ob, m, n, k, batch, da, lda, strideA, 1, db, ldb, strideB, 1, dc, ldc, strideC,
              mk<R>((R)alpha[0], (R)alpha[1]), mk<R>((R)beta[0], (R)beta[1]));
      HIPCHK(hipMemcpyAsync(hc.data(), dc, nc * sizeof(Cx), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (long i = 0; i < nc; ++i) {
        C[2 * i] = hc[i].x;
        C[2 * i + 1] = hc[i].y;
      }
    };
    if (prec == PHX_FP64) run(double());
    else run(float());
    return PHX_OK;
  });
}

int phx_small_orth(phx_ctx* ctx, int m, int batch, const double* G, double drop, double* C0, int* keep) {
  return guard(ctx, [&]() {
    if (m < 1 || m > 64 || batch < 1 || !G || !C0 || !keep || !(drop > 0)) fail(ctx, PHX_EINVAL, "bad arguments");
    hipStream_t st = ctx->stream;
    const long n = (long)m * m * batch;
    double2* dg = dbuf<double2>(ctx, "tA", n);
    double2* dc = dbuf<double2>(ctx, "tB", n);
    int* dk = dbuf<int>(ctx, "tK", (long)m * batch);
    HIPCHK(hipMemcpyAsync(dg, G, n * sizeof(double2), hipMemcpyHostToDevice, st));
    launch_chol_drop(dg, m, batch, drop, dc, dk, st);
    KCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(C0, dc, n * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(keep, dk, (long)m * batch * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PHX_OK;
  });
}

int phx_small_eig(phx_ctx* ctx, int m, int s, int batch, const double* G, const int* keep, double* C,
                  double* theta) {
  return guard(ctx, [&]() {
    if (m < 1 || m > 64 || s < 1 || s > m || batch < 1 || !G || !keep || !C || !theta)
      fail(ctx, PHX_EINVAL, "bad arguments");
    hipStream_t st = ctx->stream;
    const long n = (long)m * m * batch;
    double2* dg = dbuf<double2>(ctx, "tA", n);
    double2* dc = dbuf<double2>(ctx, "tB", (long)m * s * batch);
    int* dk = dbuf<int>(ctx, "tK", (long)m * batch);
    double* dt = dbuf<double>(ctx, "tT", (long)s * batch);
    HIPCHK(hipMemcpyAsync(dg, G, n * sizeof(double2), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dk, keep, (long)m * batch * sizeof(int), hipMemcpyHostToDevice, st));
    launch_rr_eig(dg, dk, m, s, batch, dc, dt, nullptr, st);
    KCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(C, dc, (long)m * s * batch * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(theta, dt, (long)s * batch * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PHX_OK;
  });
}

int phx_small_rr(phx_ctx* ctx, int m, int s, int batch, const double* G2, double drop, double* Cx, double* Cp,
                 double* theta, int* keep) {
  return guard(ctx, [&]() {
    if (m < 1 || m > 64 || s < 1 || s > m || batch < 1 || !G2 || !Cx || !Cp || !theta || !keep || !(drop > 0))
      fail(ctx, PHX_EINVAL, "bad arguments");
    hipStream_t st = ctx->stream;
    const long n2 = 2L * m * m * batch, ns = (long)m * s * batch;
    double2* dg = dbuf<double2>(ctx, "tA", n2);
    double2* dc0 = dbuf<double2>(ctx, "tB", (long)m * m * batch);
    double2* dx = dbuf<double2>(ctx, "tC", ns);
    double2* dp = dbuf<double2>(ctx, "tD", ns);
    int* dk = dbuf<int>(ctx, "tK", (long)m * batch);
    double* dt = dbuf<double>(ctx, "tT", (long)s * batch);
    HIPCHK(hipMemcpyAsync(dg, G2, n2 * sizeof(double2), hipMemcpyHostToDevice, st));
    launch_rr_gen(dg, m, s, batch, drop, dc0, dk, dx, dp, dt, nullptr, st, nullptr, 0, ctx->opt.small_eig);
    KCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(Cx, dx, ns * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(Cp, dp, ns * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(theta, dt, (long)s * batch * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(keep, dk, (long)m * batch * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PHX_OK;
  });
}

int phx_zposv(phx_ctx* ctx, phx_precision prec, int n, int nrhs, int batch, const double* A, double* B) {
  return guard(ctx, [&]() {
    if (n < 64 || n % 64 || nrhs < 1 || batch < 1 || !A || !B) fail(ctx, PHX_EINVAL, "bad zposv arguments");
    hipStream_t st = ctx->stream;
    const long na = (long)n * n * batch, nb = (long)n * nrhs * batch;
    auto run = [&](auto tag) {
      typedef decltype(tag) R;
      typedef C_t<R> Cx;
      std::vector<Cx> ha(na), hb(nb);
      for (long i = 0; i < na; ++i) ha[i] = mk<R>((R)A[2 * i], (R)A[2 * i + 1]);
      for (long i = 0; i < nb; ++i) hb[i] = mk<R>((R)B[2 * i], (R)B[2 * i + 1]);
      Cx* da = dbuf<Cx>(ctx, "tA", na);
      Cx* db = dbuf<Cx>(ctx, "tB", nb);
      Cx* dz = dbuf<Cx>(ctx, "tC", nb);
      Cx* dinv = dbuf<Cx>(ctx, "tD", (long)batch * (n / 64) * 4096);
      HIPCHK(hipMemcpyAsync(da, ha.data(), na * sizeof(Cx), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(db, hb.data(), nb * sizeof(Cx), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemsetAsync(ctx->dflag, 0, sizeof(int), st));
      KCHK(potrf_batched<R>(da, n, n, (long)n * n, batch, dinv, (long)(n / 64) * 4096, ctx->dflag, st));
      Cx* sbi = nullptr;
      if (ctx->opt.sbinv) {
        const long ws = sizeof(R) == 4 ? 256 : 128;
        sbi = dbuf<Cx>(ctx, "tS", (long)batch * ((n + ws - 1) / ws) * ws * ws);
        Cx* sbw = dbuf<Cx>(ctx, "tW", (long)batch * ((n + ws - 1) / ws) * (ws * ws + ws * ws / 4));
        KCHK(sb_inverse_batched<R>(da, n, n, (long)n * n, batch, dinv, (long)(n / 64) * 4096, sbi, sbw, st));
      }
      KCHK(potrs_batched<R>(da, n, n, (long)n * n, batch, dinv, (long)(n / 64) * 4096, db, n, (long)n * nrhs, dz, n,
                            (long)n * nrhs, nrhs, st, nullptr, sbi));
      int flag = 0;
      HIPCHK(hipMemcpyAsync(&flag, ctx->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(hb.data(), db, nb * sizeof(Cx), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      if (flag) fail(ctx, PHX_ENOTPD, "matrix is not positive definite");
      for (long i = 0; i < nb; ++i) {
        B[2 * i] = hb[i].x;
        B[2 * i + 1] = hb[i].y;
      }
    };
    if (prec == PHX_FP64) run(double());
    else run(float());
    return PHX_OK;
  });
}

// ------------------------------------------------------------------ design projection

static long check_projection(phx_ctx* ctx, const phx_projection* p) {
  long nd = 0;
  if (const char* e = phx_host::check_projection(p, &nd)) fail(ctx, PHX_EINVAL, e);
  return nd;
}

int phx_project_dev(phx_ctx* ctx, const phx_projection* p, const double* x_dev, double* rho_dev, void* stream) {
  return guard(ctx, [&]() {
    check_projection(ctx, p);
    if (!x_dev || !rho_dev) fail(ctx, PHX_EINVAL, "x_dev or rho_dev is NULL");
    if (stream) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    launch_project(p->nv, p->spacing, p->radius, p->beta, p->octant, x_dev, rho_dev, ctx->stream);
    KCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return PHX_OK;
  });
}

int phx_project_adjoint_dev(phx_ctx* ctx, const phx_projection* p, const double* x_dev, const double* grad_rho_dev,
                            double* grad_x_dev, void* stream) {
  return guard(ctx, [&]() {
    check_projection(ctx, p);
    if (!x_dev || !grad_rho_dev || !grad_x_dev) fail(ctx, PHX_EINVAL, "a device pointer is NULL");
    if (stream) HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    const long ne = (long)p->nv * p->nv * p->nv;
    double* coef = dbuf<double>(ctx, "proj_coef", ne);
    launch_project_adjoint(p->nv, p->spacing, p->radius, p->beta, p->octant, x_dev, grad_rho_dev, coef, grad_x_dev,
                           ctx->stream);
    KCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return PHX_OK;
  });
}

int phx_project_adjoint_dev_noalloc(phx_ctx* ctx, const phx_projection* p, const double* x_dev,
                                    const double* grad_rho_dev, double* grad_x_dev, void* stream) {
  return guard(ctx, [&]() {
    check_projection(ctx, p);
    if (!x_dev || !grad_rho_dev || !grad_x_dev) fail(ctx, PHX_EINVAL, "a device pointer is NULL");
    const long ne = (long)p->nv * p->nv * p->nv;
    if (ne > NOALLOC_SCRATCH_DOUBLES)
      fail(ctx, PHX_EINVAL, "nv^3 exceeds the allocation-free scratch (nv <= 64); use phx_project_adjoint_dev");
    double* coef = scratch_addr(ctx->device);
    if (!coef) fail(ctx, PHX_EHIP, "the device scratch of this GPU was not set up");
    // every element's coefficient is written before the second kernel reads it: nothing to clear
    launch_project_adjoint(p->nv, p->spacing, p->radius, p->beta, p->octant, x_dev, grad_rho_dev, coef, grad_x_dev,
                           stream ? (hipStream_t)stream : ctx->stream);
    KCHK(hipGetLastError());
    return PHX_OK;
  });
}

int phx_project(phx_ctx* ctx, const phx_projection* p, const double* x, double* rho) {
  return guard(ctx, [&]() {
    const long nx = check_projection(ctx, p);
    if (!x || !rho) fail(ctx, PHX_EINVAL, "x or rho is NULL");
    const long ne = (long)p->nv * p->nv * p->nv;
    double* xd = dbuf<double>(ctx, "proj_x", nx);
    double* rd = dbuf<double>(ctx, "proj_rho", ne);
    HIPCHK(hipMemcpyAsync(xd, x, nx * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    launch_project(p->nv, p->spacing, p->radius, p->beta, p->octant, xd, rd, ctx->stream);
    KCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(rho, rd, ne * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return PHX_OK;
  });
}

int phx_project_adjoint(phx_ctx* ctx, const phx_projection* p, const double* x, const double* grad_rho,
                        double* grad_x) {
  return guard(ctx, [&]() {
    const long nx = check_projection(ctx, p);
    if (!x || !grad_rho || !grad_x) fail(ctx, PHX_EINVAL, "a pointer is NULL");
    const long ne = (long)p->nv * p->nv * p->nv;
    double* xd = dbuf<double>(ctx, "proj_x", nx);
    double* gd = dbuf<double>(ctx, "proj_grho", ne);
    double* coef = dbuf<double>(ctx, "proj_coef", ne);
    double* gx = dbuf<double>(ctx, "proj_gx", nx);
    HIPCHK(hipMemcpyAsync(xd, x, nx * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(gd, grad_rho, ne * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    launch_project_adjoint(p->nv, p->spacing, p->radius, p->beta, p->octant, xd, gd, coef, gx, ctx->stream);
    KCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(grad_x, gx, nx * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return PHX_OK;
  });
}

}  // extern "C"
