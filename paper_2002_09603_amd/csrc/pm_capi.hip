// C ABI entry points (include/poromech.h): argument validation, context
// lifetime, timing, and conversion of internal errors to return codes.
#include <chrono>
#include <exception>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstring>

#include "pm_internal.h"

using pm::Error;

namespace {

thread_local std::string g_setup_error = "no error";

// y = d .* x
__global__ void k_diag_mul(int64_t n, const double* __restrict__ d, const double* __restrict__ x,
                           double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = d[i] * x[i];
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int g_live_contexts = 0;

// Scratch of pm_solve_noalloc: the FGMRES workspace (basis, preconditioned
// vectors, reduction partials, device scalars) of callers that cannot
// allocate.  One copy per GPU, held until the process ends; its device
// address comes from hipGetSymbolAddress (never the host-side name).
constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kNoallocMaxRestart = 64;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of the current device's scratch, looked up once per device
// (pm_setup calls this with the context's device current).
void* scratch_base() {
  int dev = 0;
  PM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(PM_EINTERNAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(PM_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

template <class F>
int guarded(pm_ctx* c, F&& f) {
  if (c) pm::set_alloc_stream(c->s);
  try {
    return f();
  } catch (const Error& e) {
    if (c) c->err = e.what();
    return e.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return PM_EINTERNAL;
  }
}

void free_ctx_buffers(pm_ctx* c) {
  using pm::dfree;
  for (void* p : {(void*)c->coords, (void*)c->E, (void*)c->kappa, (void*)c->Ke, (void*)c->ae, (void*)c->vol,
                  (void*)c->Minv, (void*)c->Mp, (void*)c->Mb, (void*)c->Mq, (void*)c->g, (void*)c->alpha, (void*)c->stabw, (void*)c->bp, (void*)c->auu_diag,
                  (void*)c->ufix, (void*)c->pifix, (void*)c->status, (void*)c->V, (void*)c->Z, (void*)c->Zf, (void*)c->wvec,
                  (void*)c->rvec, (void*)c->xvec, (void*)c->red, (void*)c->hcol, (void*)c->pw64, (void*)c->pw32,
                  (void*)c->mfe_lq, (void*)c->mfe_dqinv, (void*)c->mfe_work})
    dfree(p);
  if (c->hhost) (void)hipHostFree(c->hhost);
  c->Auu.free_all();
  c->Cpi.free_all();
  c->Cp.free_all();
  c->Hu.free_all();
  c->Hpi.free_all();
  c->Hcp.free_all();
  c->lat.free_all();
  c->cpi.free_all();
  for (hipStream_t* ps : {&c->s_side_u, &c->s_side_pi})
    if (*ps) {
      (void)hipStreamSynchronize(*ps);
      (void)hipStreamDestroy(*ps);
      *ps = nullptr;
    }
  if (c->s_aux) {
    (void)hipStreamSynchronize(c->s_aux);
    (void)hipStreamDestroy(c->s_aux);
    c->s_aux = nullptr;
  }
}

void copy_in(pm_ctx* c, double* dst, const double* src, int64_t n) {
  PM_HIP(hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDefault, c->s));
}

// validates positivity of a device field (host copy; setup-time only)
void check_positive(pm_ctx* c, const double* dev, int64_t n, const char* what) {
  std::vector<double> h(n);
  PM_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double) * n, hipMemcpyDeviceToHost, c->s));
  PM_HIP(hipStreamSynchronize(c->s));
  for (int64_t i = 0; i < n; ++i)
    if (!(h[i] > 0.0) || !std::isfinite(h[i]))
      throw Error(PM_EINVAL, std::string(what) + " must be positive and finite (index " + std::to_string(i) + ")");
}

pm::AmgParams params_u(const pm_ctx* c) {
  pm::AmgParams p;
  p.theta = c->opts.theta_u;
  p.coarse_max = c->opts.coarse_max;
  p.cheb_degree = c->opts.cheb_degree;
  p.cycles = c->opts.cycles_u;
  p.agg_dist = c->opts.agg_dist_u;
  p.cheb_lower = c->opts.cheb_lower;
  p.fp32 = c->opts.precond_fp32 != 0;
  p.p_trunc = c->opts.p_trunc_u;
  p.side = c->s_side_u;
  p.rbm = c->opts.rbm_u != 0;
  p.coords = c->coords;
  return p;
}

pm::AmgParams params_pi(const pm_ctx* c) {
  pm::AmgParams p = params_u(c);
  p.rbm = false;
  p.theta = c->opts.theta_pi;
  p.coarse_max = c->opts.coarse_max * 3;
  p.cheb_degree = c->opts.cheb_degree_pi;
  p.cycles = c->opts.cycles_pi;
  p.agg_dist = c->opts.agg_dist_pi;
  p.p_trunc = c->opts.p_trunc_pi;
  if (c->opts.cheb_lower_pi > 0.0) p.cheb_lower = c->opts.cheb_lower_pi;
  p.side = c->s_side_pi;
  return p;
}

// the MFE preconditioner's C~_p hierarchy: the C~_pi settings (V-cycles per
// application included), FP64 levels, on the caller's stream
pm::AmgParams params_cp(const pm_ctx* c) {
  pm::AmgParams p = params_pi(c);
  p.fp32 = false;
  p.side = nullptr;
  return p;
}

// C~_p, its hierarchy and the A_qq sweep data, once per assembly and dt
void ensure_mfe_prec(pm_ctx* c) {
  if (!c->mfe_valid) pm::mfe_prec_setup(c, params_cp(c));
}

// B~_p, C~_pi (assembled and packed per cell) and C~_pi's AMG hierarchy, on
// stream s (the caller's thread must have made s its allocation stream)
void setup_pi(pm_ctx* c, hipStream_t s) {
  const pm::Grid G = pm::grid_of(c);
  pm::build_cpi(c, s);
  if (c->opts.cell_pi) pm::cellpi_build(c, s);
  pm::amg_setup(s, c->Cpi, params_pi(c), c->Hpi, nullptr, &G, c->opts.cell_pi ? &c->cpi : nullptr);
}

// The two hierarchies are independent: A_uu's is built on the caller's
// stream by this thread while C~_pi's is built on the library's second
// stream by a helper thread (the set-up is dominated by small kernels and
// host round trips for sizes, which the two overlap).  Both start after the
// assembly has completed on the caller's stream and both streams are
// synchronized before this returns; each hierarchy's result does not depend
// on the interleaving.
void setup_hierarchies(pm_ctx* c, bool with_u) {
  // with_u: after assemble_all; the A_uu values are filled on this thread
  // (assemble_auu) while the helper thread builds C~_pi, which needs only
  // the A_uu diagonal
  if (with_u) {
    PM_HIP(hipStreamSynchronize(c->s));
    if (!c->s_aux) PM_HIP(hipStreamCreateWithFlags(&c->s_aux, hipStreamNonBlocking));
    if (!c->s_side_u) PM_HIP(hipStreamCreateWithFlags(&c->s_side_u, hipStreamNonBlocking));
    if (!c->s_side_pi) PM_HIP(hipStreamCreateWithFlags(&c->s_side_pi, hipStreamNonBlocking));
    int dev = 0;
    PM_HIP(hipGetDevice(&dev));
    std::exception_ptr pi_err;
    std::thread th([c, dev, &pi_err] {
      try {
        PM_HIP(hipSetDevice(dev));
        pm::set_alloc_stream(c->s_aux);
        setup_pi(c, c->s_aux);
        PM_HIP(hipStreamSynchronize(c->s_aux));
      } catch (...) {
        pi_err = std::current_exception();
      }
    });
    hipEvent_t fill0 = nullptr, fill1 = nullptr;
    try {
      const pm::Grid G = pm::grid_of(c);
      PM_HIP(hipEventCreate(&fill0));
      PM_HIP(hipEventCreate(&fill1));
      PM_HIP(hipEventRecord(fill0, c->s));
      pm::assemble_auu(c);
      PM_HIP(hipEventRecord(fill1, c->s));
      pm::amg_setup(c->s, c->Auu, params_u(c), c->Hu, c->lattice ? &c->lat : nullptr, &G);
    } catch (...) {
      th.join();
      if (fill0) (void)hipEventDestroy(fill0);
      if (fill1) (void)hipEventDestroy(fill1);
      throw;
    }
    th.join();
    // the A_uu values are assembly: their time on the caller's stream moves from
    // the set-up to the assembly figure (it overlaps the C~_pi set-up)
    float fill_ms = 0.0f;
    const hipError_t ev = hipEventElapsedTime(&fill_ms, fill0, fill1);
    (void)hipEventDestroy(fill0);
    (void)hipEventDestroy(fill1);
    if (pi_err) std::rethrow_exception(pi_err);
    PM_HIP(ev);
    c->fill_s = 1e-3 * fill_ms;
    c->hier_u_ok = true;
  } else {
    setup_pi(c, c->s);
  }
  c->info.levels_u = (int)c->Hu.L.size();
  c->info.levels_pi = (int)c->Hpi.L.size();
  c->info.opcx_u = c->Hu.opcx;
  c->info.opcx_pi = c->Hpi.opcx;
  c->info.lattice_uu = c->lattice ? 1 : 0;
  c->info.lattice_form = !c->lattice ? 0 : c->lat.cube ? 3 : c->lat.sym ? 2 : 1;
  c->info.block_minv = c->mblock ? 1 : 0;
  c->info.ncoarse_u = c->Hu.ncoarse;
  c->info.ncoarse_pi = c->Hpi.ncoarse;
}

void assemble_and_setup(pm_ctx* c) {
  PM_HIP(hipStreamSynchronize(c->s));
  const double t0 = now_s();
  if (!c->lattice) c->Ke = pm::dalloc<double>(576 * c->nc);
  try {
    pm::assemble_all(c);
  } catch (...) {
    pm::dfree(c->Ke);
    c->Ke = nullptr;
    throw;
  }
  PM_HIP(hipStreamSynchronize(c->s));
  const double t1 = now_s();
  try {
    setup_hierarchies(c, true);
  } catch (...) {
    pm::dfree(c->Ke);
    c->Ke = nullptr;
    throw;
  }
  PM_HIP(hipStreamSynchronize(c->s));
  pm::dfree(c->Ke);
  c->Ke = nullptr;
  const double t2 = now_s();
  c->info.t_asm = (t1 - t0) + c->fill_s;
  c->info.t_setup = (t2 - t1) - c->fill_s;
  c->assembled = true;
}

}  // namespace

extern "C" {

void pm_default_opts(pm_opts* o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->restart = 100;
  o->max_it = 1000;
  o->precond_fp32 = 0;
  o->stabilize = 1;
  o->increment_stab = 1;
  o->cheb_degree = 2;
  o->coarse_max = 64;
  o->cheb_degree_pi = 2;
  o->cycles_u = 1;
  o->cycles_pi = 1;
  o->orth_passes = 2;
  o->theta_u = 0.0;
  o->agg_dist_u = 2;
  o->agg_dist_pi = 2;
  o->cheb_lower = 0.3;
  o->rtol_transpose = 0.0;
  o->restart_transpose = 100;
  o->orth_passes_transpose = 2;
  o->lattice_uu = 1;
  o->p_trunc_pi = 0.02;
  o->p_trunc_u = 0.02;
  o->cheb_lower_pi = 0.0;
  o->cell_pi = 1;
  o->theta_pi = 0.08;
  o->block_minv = 1;
  o->rbm_u = 0;
}

int pm_setup(const pm_mesh* mesh, const pm_material* mat, const pm_bc* bc, double dt, const pm_opts* opts,
             void* stream, pm_ctx** out) {
  if (!out) {
    g_setup_error = "pm_setup: out is NULL";
    return PM_EINVAL;
  }
  *out = nullptr;
  pm_ctx* c = new (std::nothrow) pm_ctx();
  if (!c) {
    g_setup_error = "pm_setup: host allocation failed";
    return PM_ENOMEM;
  }
  const int rc = guarded(c, [&]() -> int {
    if (!mesh || !mat || !bc) throw Error(PM_EINVAL, "pm_setup: mesh, material and bc are required");
    if (mesh->nx < 2 || mesh->ny < 2 || mesh->nz < 2 || (mesh->nx & 1) || (mesh->ny & 1) || (mesh->nz & 1))
      throw Error(PM_EINVAL, "pm_setup: nx, ny, nz must be even and >= 2 (2x2x2 macro-elements)");
    if (!mat->E || !mat->kappa) throw Error(PM_EINVAL, "pm_setup: E and kappa are required");
    if (!(mat->nu > 0.0 && mat->nu < 0.5)) throw Error(PM_EINVAL, "pm_setup: nu must lie in (0, 0.5)");
    if (!(mat->mu > 0.0) || !(mat->S_eps >= 0.0) || !std::isfinite(mat->biot))
      throw Error(PM_EINVAL, "pm_setup: mu > 0, S_eps >= 0 and a finite Biot coefficient are required");
    if (!(dt > 0.0) || !std::isfinite(dt)) throw Error(PM_EINVAL, "pm_setup: dt must be positive");
    if (bc->kind != PM_BC_COLUMN && bc->kind != PM_BC_ROLLERS && bc->kind != PM_BC_CANTILEVER)
      throw Error(PM_EINVAL, "pm_setup: unknown bc kind");
    c->s = (hipStream_t)stream;
    pm::set_alloc_stream(c->s);
    c->nx = mesh->nx;
    c->ny = mesh->ny;
    c->nz = mesh->nz;
    const int64_t nx = c->nx, ny = c->ny, nz = c->nz;
    c->nn = (nx + 1) * (ny + 1) * (nz + 1);
    c->nc = nx * ny * nz;
    c->nfx = (nx + 1) * ny * nz;
    c->nfy = nx * (ny + 1) * nz;
    c->nfz = nx * ny * (nz + 1);
    c->nf = c->nfx + c->nfy + c->nfz;
    if (c->nf >= ((int64_t)1 << 31) || c->nn >= ((int64_t)1 << 31))
      throw Error(PM_EINVAL, "pm_setup: meshes with 2^31 or more faces or nodes are not supported");
    c->nmacro = c->nc / 8;
    c->n_u = 3 * c->nn;
    c->n_p = c->nc;
    c->n_pi = c->nf;
    c->N = c->n_u + c->n_p + c->n_pi;
    if (c->N >= ((int64_t)1 << 31) / 9) throw Error(PM_EINVAL, "pm_setup: problem too large for 32-bit indices");
    c->nu = mat->nu;
    c->biot = mat->biot;
    c->S = mat->S_eps;
    c->mu = mat->mu;
    c->dt = dt;
    for (int d = 0; d < 3; ++d) c->trac[d] = bc->traction_top[d];
    c->p_top = bc->p_top;
    c->bc_kind = bc->kind;
    if (opts) c->opts = *opts; else pm_default_opts(&c->opts);
    if (c->opts.restart < 1 || c->opts.max_it < 1 || c->opts.cheb_degree < 1 || c->opts.coarse_max < 1 ||
        c->opts.cheb_degree_pi < 1 || c->opts.cycles_u < 1 || c->opts.cycles_pi < 1 || c->opts.cycles_u > 8 ||
        c->opts.cycles_pi > 8 || c->opts.orth_passes < 1 || c->opts.orth_passes > 2 || !(c->opts.rtol > 0.0) ||
        c->opts.agg_dist_u < 1 || c->opts.agg_dist_u > 2 || c->opts.agg_dist_pi < 1 || c->opts.agg_dist_pi > 2 ||
        !(c->opts.cheb_lower > 0.0 && c->opts.cheb_lower < 1.0) || c->opts.restart > 500 ||
        c->opts.restart_transpose < 0 || c->opts.restart_transpose > 500 || c->opts.orth_passes_transpose < 0 ||
        c->opts.orth_passes_transpose > 2 || !(c->opts.rtol_transpose >= 0.0) ||
        !(c->opts.p_trunc_pi >= 0.0 && c->opts.p_trunc_pi < 1.0) ||
        !(c->opts.p_trunc_u >= 0.0 && c->opts.p_trunc_u < 1.0) ||
        !(c->opts.cheb_lower_pi >= 0.0 && c->opts.cheb_lower_pi < 1.0))
      throw Error(PM_EINVAL, "pm_setup: invalid solver options");
    c->coords = pm::dalloc<double>(3 * c->nn);
    c->E = pm::dalloc<double>(c->nc);
    c->kappa = pm::dalloc<double>(3 * c->nc);
    if (mesh->coords) {
      copy_in(c, c->coords, mesh->coords, 3 * c->nn);
    } else {
      if (!(mesh->Lx > 0 && mesh->Ly > 0 && mesh->Lz > 0)) throw Error(PM_EINVAL, "pm_setup: box size must be positive");
      std::vector<double> X(3 * c->nn);
      for (int64_t k = 0; k <= nz; ++k)
        for (int64_t j = 0; j <= ny; ++j)
          for (int64_t i = 0; i <= nx; ++i) {
            const int64_t n = i + (nx + 1) * (j + (ny + 1) * k);
            X[3 * n + 0] = mesh->Lx * (double)i / (double)nx;
            X[3 * n + 1] = mesh->Ly * (double)j / (double)ny;
            X[3 * n + 2] = mesh->Lz * (double)k / (double)nz;
          }
      PM_HIP(hipMemcpyAsync(c->coords, X.data(), sizeof(double) * X.size(), hipMemcpyHostToDevice, c->s));
      PM_HIP(hipStreamSynchronize(c->s));
    }
    copy_in(c, c->E, mat->E, c->nc);
    copy_in(c, c->kappa, mat->kappa, 3 * c->nc);
    check_positive(c, c->E, c->nc, "E");
    check_positive(c, c->kappa, 3 * c->nc, "kappa");
    // the lattice kernels address neighbours by 32-bit byte offsets
    if (c->opts.lattice_uu && 3 * c->nn * (int64_t)sizeof(double) < (int64_t)UINT32_MAX) {
      double dev = 0.0, hmin = 0.0;
      pm::lattice_deviation(c->s, pm::grid_of(c), c->coords, &dev, &hmin);
      c->lattice = dev <= 1e-12 * hmin;
    }
    c->ae = pm::dalloc<double>(24 * c->nc);
    c->vol = pm::dalloc<double>(c->nc);
    c->Minv = pm::dalloc<double>(36 * c->nc);
    c->g = pm::dalloc<double>(6 * c->nc);
    c->alpha = pm::dalloc<double>(c->nc);
    c->stabw = pm::dalloc<double>(c->nmacro);
    c->bp = pm::dalloc<double>(c->nc);
    c->auu_diag = pm::dalloc<double>(c->n_u);
    c->ufix = pm::dalloc<uint8_t>(c->n_u);
    c->pifix = pm::dalloc<uint8_t>(c->n_pi);
    c->status = pm::dalloc<int>(1);
    (void)scratch_base();  // device address of this GPU's pm_solve_noalloc scratch, once per device
    pm::krylov_preload(c->s);
    c->wvec = pm::dalloc<double>(c->N);
    c->rvec = pm::dalloc<double>(c->N);
    c->xvec = pm::dalloc<double>(c->N);
    c->pw64 = pm::dalloc<double>(c->N);
    if (c->opts.precond_fp32) c->pw32 = pm::dalloc<float>(3 * c->N);
    return PM_OK;
  });
  if (rc != PM_OK) {
    g_setup_error = c->err;
    free_ctx_buffers(c);
    delete c;
    return rc;
  }
  *out = c;
  ++g_live_contexts;
  return PM_OK;
}

int pm_assemble(pm_ctx* c) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    assemble_and_setup(c);
    return PM_OK;
  });
}

int pm_set_dt(pm_ctx* c, double dt) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!(dt > 0.0) || !std::isfinite(dt)) throw Error(PM_EINVAL, "pm_set_dt: dt must be positive");
    c->dt = dt;
    c->mfe_valid = false;
    if (!c->assembled) return PM_OK;
    PM_HIP(hipStreamSynchronize(c->s));
    const double t0 = now_s();
    setup_hierarchies(c, false);
    PM_HIP(hipStreamSynchronize(c->s));
    c->info.t_setup = now_s() - t0;
    return PM_OK;
  });
}

int pm_update_material(pm_ctx* c, const double* E, const double* kappa) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (E) {
      copy_in(c, c->E, E, c->nc);
      check_positive(c, c->E, c->nc, "E");
    }
    if (kappa) {
      copy_in(c, c->kappa, kappa, 3 * c->nc);
      check_positive(c, c->kappa, 3 * c->nc, "kappa");
    }
    assemble_and_setup(c);
    return PM_OK;
  });
}

int pm_build_rhs(pm_ctx* c, const double* u_prev, const double* p_prev, double* b) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!b) throw Error(PM_EINVAL, "pm_build_rhs: b is NULL");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_build_rhs: call pm_assemble first");
    pm::build_rhs(c, u_prev, p_prev, b);
    return PM_OK;
  });
}

static int solve_common(pm_ctx* c, const double* b, double* u, double* pi, double* p, pm_info* info, bool tr) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!b) throw Error(PM_EINVAL, "pm_solve: b is NULL");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_solve: call pm_assemble first");
    PM_HIP(hipStreamSynchronize(c->s));
    const double t0 = now_s();
    pm_info li = c->info;
    const pm_opts saved = c->opts;
    if (tr) {
      if (c->opts.rtol_transpose > 0.0) c->opts.rtol = c->opts.rtol_transpose;
      if (c->opts.restart_transpose > 0) c->opts.restart = c->opts.restart_transpose;
      if (c->opts.orth_passes_transpose > 0) c->opts.orth_passes = c->opts.orth_passes_transpose;
    }
    int rc;
    try {
      rc = pm::fgmres(c, b, c->xvec, tr, &li);
    } catch (...) {
      c->opts = saved;
      throw;
    }
    c->opts = saved;
    if (u) PM_HIP(hipMemcpyAsync(u, c->xvec, sizeof(double) * c->n_u, hipMemcpyDeviceToDevice, c->s));
    if (p) PM_HIP(hipMemcpyAsync(p, c->xvec + c->n_u, sizeof(double) * c->n_p, hipMemcpyDeviceToDevice, c->s));
    if (pi)
      PM_HIP(hipMemcpyAsync(pi, c->xvec + c->n_u + c->n_p, sizeof(double) * c->n_pi, hipMemcpyDeviceToDevice, c->s));
    PM_HIP(hipStreamSynchronize(c->s));
    li.t_solve = now_s() - t0;
    c->info = li;
    if (info) *info = li;
    if (rc == PM_ENOCONV) c->err = "FGMRES reached max_it before rtol";
    return rc;
  });
}

int pm_solve(pm_ctx* c, const double* b, double* u, double* pi, double* p, pm_info* info) {
  return solve_common(c, b, u, pi, p, info, false);
}

int pm_solve_noalloc(pm_ctx* c, const double* b, double* u, double* pi, double* p, pm_info* info) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!b) throw Error(PM_EINVAL, "pm_solve_noalloc: b is NULL");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_solve_noalloc: call pm_assemble first");
    const int m = c->opts.restart;
    if (m > kNoallocMaxRestart)
      throw Error(PM_EINVAL, "pm_solve_noalloc: restart " + std::to_string(m) + " exceeds " +
                                 std::to_string(kNoallocMaxRestart));
    const pm::KrylovOps op = pm::step_ops(c, false);
    const bool z32 = c->opts.orth_passes == 1 && op.M32 != nullptr;
    const size_t need = pm::krylov_device_bytes(c->N, m, z32);
    if (need > kScratchBytes)
      throw Error(PM_EINVAL, "pm_solve_noalloc: the Krylov workspace of this problem (" + std::to_string(need) +
                                 " bytes for " + std::to_string(c->N) + " unknowns, restart " + std::to_string(m) +
                                 ") exceeds the static scratch of " + std::to_string(kScratchBytes) + " bytes");
    void* base = scratch_base();
    const pm::KrylovWs ws0 = pm::krylov_ws_in(base, kScratchBytes, c->N, m, z32);
    // host arrays of the Givens process and the read-back scalars: on this stack frame
    double H[(kNoallocMaxRestart + 1) * kNoallocMaxRestart], cs[kNoallocMaxRestart], sn[kNoallocMaxRestart],
        g[kNoallocMaxRestart + 1], y[kNoallocMaxRestart], hh[kNoallocMaxRestart + 8];
    pm::KrylovWs ws = ws0;
    ws.hhost = hh;
    pm::KrylovHost hw{kNoallocMaxRestart, H, cs, sn, g, y};
    PM_HIP(hipStreamSynchronize(c->s));
    const double t0 = now_s();
    pm_info li = c->info;
    const int rc = pm::fgmres_ws(c, op, ws, hw, b, c->xvec, &li);
    if (u) PM_HIP(hipMemcpyAsync(u, c->xvec, sizeof(double) * c->n_u, hipMemcpyDeviceToDevice, c->s));
    if (p) PM_HIP(hipMemcpyAsync(p, c->xvec + c->n_u, sizeof(double) * c->n_p, hipMemcpyDeviceToDevice, c->s));
    if (pi)
      PM_HIP(hipMemcpyAsync(pi, c->xvec + c->n_u + c->n_p, sizeof(double) * c->n_pi, hipMemcpyDeviceToDevice, c->s));
    PM_HIP(hipStreamSynchronize(c->s));
    li.t_solve = now_s() - t0;
    c->info = li;
    if (info) *info = li;
    if (rc == PM_ENOCONV) c->err = "FGMRES reached max_it before rtol";
    return rc;
  });
}

int pm_solve_transpose(pm_ctx* c, const double* g, double* lu, double* lpi, double* lp, pm_info* info) {
  return solve_common(c, g, lu, lpi, lp, info, true);
}

int pm_build_rhs_mfe(pm_ctx* c, const double* u_prev, const double* p_prev, double* b) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!b) throw Error(PM_EINVAL, "pm_build_rhs_mfe: b is NULL");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_build_rhs_mfe: call pm_assemble first");
    pm::build_rhs_mfe(c, u_prev, p_prev, b);
    return PM_OK;
  });
}

int pm_solve_mfe(pm_ctx* c, const double* b, double* u, double* q, double* p, pm_info* info) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!b) throw Error(PM_EINVAL, "pm_solve_mfe: b is NULL");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_solve_mfe: call pm_assemble first");
    PM_HIP(hipStreamSynchronize(c->s));
    const double t0 = now_s();
    const bool built = !c->mfe_valid;
    ensure_mfe_prec(c);
    PM_HIP(hipStreamSynchronize(c->s));
    const double t1 = now_s();
    pm::KrylovOps op;
    op.A64 = [c](const double* z, double* w) { pm::apply_mfe(c, z, w); };
    op.M64 = [c](const double* v, double* z) { pm::apply_btp(c, v, z); };
    pm_info li = c->info;
    const int rc = pm::fgmres_with(c, op, b, c->xvec, &li);
    const int64_t nq = c->n_pi;
    if (u) PM_HIP(hipMemcpyAsync(u, c->xvec, sizeof(double) * c->n_u, hipMemcpyDeviceToDevice, c->s));
    if (q) PM_HIP(hipMemcpyAsync(q, c->xvec + c->n_u, sizeof(double) * nq, hipMemcpyDeviceToDevice, c->s));
    if (p) PM_HIP(hipMemcpyAsync(p, c->xvec + c->n_u + nq, sizeof(double) * c->n_p, hipMemcpyDeviceToDevice, c->s));
    PM_HIP(hipStreamSynchronize(c->s));
    li.t_solve = now_s() - t1;
    if (built) li.t_setup = t1 - t0;  // the C~_p hierarchy; the A_uu one is pm_assemble's
    li.levels_pi = (int)c->Hcp.L.size();
    li.opcx_pi = c->Hcp.opcx;
    li.ncoarse_pi = c->Hcp.ncoarse;
    if (info) *info = li;
    if (rc == PM_ENOCONV) c->err = "FGMRES reached max_it before rtol";
    return rc;
  });
}

int pm_grad(pm_ctx* c, const double* lam, const double* x, const double* p_prev, double* dlogk, double* dlogE) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!lam || !x || !dlogk || !dlogE) throw Error(PM_EINVAL, "pm_grad: NULL argument");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_grad: call pm_assemble first");
    pm::grad(c, lam, x, p_prev, dlogk, dlogE);
    return PM_OK;
  });
}

int pm_rhs_adjoint(pm_ctx* c, const double* lam, double* cvec) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!lam || !cvec) throw Error(PM_EINVAL, "pm_rhs_adjoint: NULL argument");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_rhs_adjoint: call pm_assemble first");
    pm::rhs_adjoint(c, lam, cvec);
    return PM_OK;
  });
}

int pm_reconstruct_w(pm_ctx* c, const double* p, const double* pi, double* w) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!p || !pi || !w) throw Error(PM_EINVAL, "pm_reconstruct_w: NULL argument");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_reconstruct_w: call pm_assemble first");
    pm::reconstruct_w(c, p, pi, w);
    return PM_OK;
  });
}

int pm_apply(pm_ctx* c, int which, const double* x, double* y) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (!x || !y) throw Error(PM_EINVAL, "pm_apply: NULL argument");
    if (!c->assembled) throw Error(PM_ESTATE, "pm_apply: call pm_assemble first");
    switch (which) {
      case PM_OP_AH: pm::apply_AH(c, x, y, false); break;
      case PM_OP_AHT: pm::apply_AH(c, x, y, true); break;
      case PM_OP_MINV: pm::apply_Minv(c, x, y, false); break;
      case PM_OP_MINVT: pm::apply_Minv(c, x, y, true); break;
      case PM_OP_CPI: pm::apply_csr(c, c->Cpi, x, y); break;
      case PM_OP_BP:
        k_diag_mul<<<pm::blocks_for(c->n_p), pm::kBlock, 0, c->s>>>(c->n_p, c->bp, x, y);
        PM_CHECK_LAUNCH();
        break;
      case PM_OP_AUU: pm::apply_csr(c, c->Auu, x, y); break;
      case PM_OP_VCYCLE_U: pm::amg_vcycle(c->s, c->Hu, x, y); break;
      case PM_OP_VCYCLE_PI: pm::amg_vcycle(c->s, c->Hpi, x, y); break;
      case PM_OP_MFE: pm::apply_mfe(c, x, y); break;
      case PM_OP_CP:
        ensure_mfe_prec(c);
        pm::apply_csr(c, c->Cp, x, y);
        break;
      case PM_OP_VCYCLE_CP:
        ensure_mfe_prec(c);
        pm::amg_vcycle(c->s, c->Hcp, x, y);
        break;
      case PM_OP_BTP:
        ensure_mfe_prec(c);
        pm::apply_btp(c, x, y);
        break;
      default: throw Error(PM_EINVAL, "pm_apply: unknown operator");
    }
    return PM_OK;
  });
}

int pm_profile_begin(pm_ctx* c, uint32_t mask) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (mask & ~((1u << pm::kProfCount) - 2u)) throw Error(PM_EINVAL, "pm_profile_begin: unknown kernel id in mask");
    pm::g_prof.reset(mask);
    return PM_OK;
  });
}

int pm_profile_end(pm_ctx* c, int id, int64_t* launches, double* ms, double* bytes, double* flops) {
  if (!c) return PM_EINVAL;
  return guarded(c, [&]() -> int {
    if (id < 1 || id >= pm::kProfCount || !launches || !ms || !bytes)
      throw Error(PM_EINVAL, "pm_profile_end: bad kernel id or NULL output");
    double f = 0.0;
    pm::g_prof.collect(id, launches, ms, bytes, &f);
    if (flops) *flops = f;
    return PM_OK;
  });
}

int pm_sizes(const pm_ctx* c, int64_t* out) {
  if (!c || !out) return PM_EINVAL;
  out[0] = c->n_u;
  out[1] = c->n_p;
  out[2] = c->n_pi;
  out[3] = c->N;
  out[4] = c->nn;
  out[5] = c->nmacro;
  return PM_OK;
}

int pm_get_info(const pm_ctx* c, pm_info* info) {
  if (!c || !info) return PM_EINVAL;
  *info = c->info;
  return PM_OK;
}

const char* pm_last_error(const pm_ctx* c) {
  if (!c) return g_setup_error.c_str();
  return c->err.empty() ? "no error" : c->err.c_str();
}

void pm_destroy(pm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->s);
  pm::set_alloc_stream(c->s);
  free_ctx_buffers(c);
  delete c;
  if (--g_live_contexts <= 0) {
    g_live_contexts = 0;
    pm::release_device_cache();
  }
}

}  // extern "C"

