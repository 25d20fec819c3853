// Batched preconditioned conjugate gradient for the DFPT linear systems
// (Sec. 2.3 Eq. linear_system at q = 0, the valence projector of
// Eq. projector, and the CG recurrence of Sec. 2.4, Eqs. ax1 .. updatedold),
// one system per (k-point, band), all of them advancing in the same launches
// (Sec. 3, Algorithm phonon_new).  Converged systems are frozen.
//
//   A x = H x - eps_nu S x + alpha_k SU (SU^H x),   U = occupied states at k
//   (S = 1 without an overlap; with one, SU = S U is formed once, so the
//   projector term of Eqs. compute_mu, use_mu and apply_s_ch costs two
//   small products per application, and -eps S x is accumulated into H x by
//   the overlap kernel)
//   r = A x - b;  loop:  d = M^-1 r;  rho = Re(d^H r);  stop if |rho| < thr;
//                        (from the 2nd iteration) d += (rho/rho_old) d_old;
//                        t = A d;  lambda = -Re(d^H r) / Re(d^H t);
//                        x += lambda d;  r += lambda t;  d_old = d;  rho_old = rho
//   M_GG = max(1, (|k+G|^2/2) / <u_nu|T|u_nu>)   (Sec. 2.4 preconditioner)
// The paper keeps rho, gamma and lambda on the CPU; here every scalar and
// flag stays on the device and the host only reads, one iteration late, how
// many systems are still active.  max_iter bounds the updates of the whole
// solve (both phases of the mixed mode together).
// Mixed precision applies H in complex64 (everything else FP64) until each
// system's residual has dropped by a fixed factor (or below thr), then
// recomputes r = A x - b with H in FP64 and continues to thr: the FP32 phase
// does the bulk of the work and the FP64 phase removes its error.  H is only
// applied to the systems still active.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "host_util.hpp"
#include "internal.hpp"

namespace mkpw {

using cd = cplx<double>;

namespace {

__device__ __forceinline__ double block_sum2(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// T_nu = sum_G |k+G|^2/2 |u_nu(G)|^2 for nu < nrhs
__global__ __launch_bounds__(256) void tkin_kernel(const cd* U, int nocc, const double* kin, const int* npw, int npwx,
                                                   int nrhs, double* tk) {
  const int k = blockIdx.y, nu = blockIdx.x;
  __shared__ double red[4];
  const cd* u = U + ((long)k * nocc + nu) * npwx;
  double s = 0.0;
  for (int g = threadIdx.x; g < npw[k]; g += 256) s += kin[(long)k * npwx + g] * (u[g].x * u[g].x + u[g].y * u[g].y);
  s = block_sum2(s, red);
  if (threadIdx.x == 0) tk[(long)k * nrhs + nu] = s;
}

// W(k)[mu][nu] *= alpha_k
__global__ void scale_w_kernel(cd* W, int n, const double* alpha) {
  const int k = blockIdx.x;
  const double a = alpha[k];
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    cd w = W[(long)k * n + e];
    W[(long)k * n + e] = {a * w.x, a * w.y};
  }
}

// r = t - eps x - b  (t = H x + alpha U U^H x), or r = t - b when t already
// holds the -eps S x term;  every system restarts as active
__global__ __launch_bounds__(256) void init_resid_kernel(const cd* t, const cd* x, const cd* b, const double* eps,
                                                         cd* r, int npwx, int* active, const int* npw, int nrhs,
                                                         int sub_eps) {
  const long sys = blockIdx.x;
  const int k = (int)(sys / nrhs);
  const double e = sub_eps ? eps[sys] : 0.0;
  const long o = sys * npwx;
  for (int g = threadIdx.x; g < npwx; g += 256) {
    cd v = {0.0, 0.0};
    if (g < npw[k]) v = {t[o + g].x - e * x[o + g].x - b[o + g].x, t[o + g].y - e * x[o + g].y - b[o + g].y};
    r[o + g] = v;
  }
  if (threadIdx.x == 0) active[sys] = 1;
}

// d = M^-1 r, rho = Re(d^H r); convergence when |rho| < max(thr, rel |rho at the
// phase's first iteration|); gamma step from the 2nd iteration
__global__ __launch_bounds__(256) void step1_kernel(const cd* r, cd* d, const cd* dold, const double* kin,
                                                    const double* tk, const int* npw, int npwx, int nrhs, double* rho,
                                                    double* rho_old, double* rho0, int* active, int first, double thr,
                                                    double rel, int* iters) {
  const long sys = blockIdx.x;
  if (!active[sys]) return;
  const int k = (int)(sys / nrhs);
  __shared__ double red[4];
  const long o = sys * npwx;
  const double tkin = tk[sys];
  double s = 0.0;
  for (int g = threadIdx.x; g < npw[k]; g += 256) {
    double m = fmax(1.0, kin[(long)k * npwx + g] / tkin);
    cd v = {r[o + g].x / m, r[o + g].y / m};
    s += v.x * r[o + g].x + v.y * r[o + g].y;
  }
  s = block_sum2(s, red);
  if (first && threadIdx.x == 0) rho0[sys] = s;
  if (fabs(s) < fmax(thr, rel * fabs(first ? s : rho0[sys]))) {
    if (threadIdx.x == 0) {
      active[sys] = 0;
      rho[sys] = s;
    }
    return;
  }
  const double gam = first ? 0.0 : s / rho_old[sys];
  for (int g = threadIdx.x; g < npwx; g += 256) {
    cd v = {0.0, 0.0};
    if (g < npw[k]) {
      double m = fmax(1.0, kin[(long)k * npwx + g] / tkin);
      v = {r[o + g].x / m, r[o + g].y / m};
      if (!first) v = {v.x + gam * dold[o + g].x, v.y + gam * dold[o + g].y};
    }
    d[o + g] = v;
  }
  if (threadIdx.x == 0) {
    rho[sys] = s;
    iters[sys] += 1;  // one more update for this system
  }
}

// number of nonzero flags (one workgroup)
__global__ __launch_bounds__(1024) void count_active_kernel(const int* __restrict__ a, long n, int* out) {
  __shared__ int red[16];
  int s = 0;
  for (long i = threadIdx.x; i < n; i += 1024) s += a[i] != 0;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < 16; ++w) t += red[w];
    *out = t;
  }
}

__global__ void fill_int_kernel(int* p, long n, int v) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) p[e] = v;
}

// t -= eps d (when sub_eps) ; lambda = -Re(d^H r)/Re(d^H t) ; x += lambda d ;
// r += lambda t ; d_old = d ; rho_old = rho
__global__ __launch_bounds__(256) void step2_kernel(cd* t, const cd* d, cd* dold, cd* x, cd* r, const double* eps,
                                                    const int* npw, int npwx, int nrhs, const double* rho,
                                                    double* rho_old, const int* active, int sub_eps) {
  const long sys = blockIdx.x;
  if (!active[sys]) return;
  const int k = (int)(sys / nrhs);
  __shared__ double red[4];
  const long o = sys * npwx;
  const double e = sub_eps ? eps[sys] : 0.0;
  double dr = 0.0, dt = 0.0;
  for (int g = threadIdx.x; g < npw[k]; g += 256) {
    cd tv = {t[o + g].x - e * d[o + g].x, t[o + g].y - e * d[o + g].y};
    t[o + g] = tv;
    dr += d[o + g].x * r[o + g].x + d[o + g].y * r[o + g].y;
    dt += d[o + g].x * tv.x + d[o + g].y * tv.y;
  }
  dr = block_sum2(dr, red);
  dt = block_sum2(dt, red);
  const double lam = -dr / dt;
  for (int g = threadIdx.x; g < npw[k]; g += 256) {
    cd dv = d[o + g], tv = t[o + g];
    x[o + g] = {x[o + g].x + lam * dv.x, x[o + g].y + lam * dv.y};
    r[o + g] = {r[o + g].x + lam * tv.x, r[o + g].y + lam * tv.y};
    dold[o + g] = dv;
  }
  if (threadIdx.x == 0) rho_old[sys] = rho[sys];
}

}  // namespace


pw_status dfpt_cg_run(pw_ctx* c, pw_prec prec, int nocc, const cd* U, const double* eps_h, const double* alpha_h,
                      int nrhs, const cd* b, cd* x, double thr, int max_iter, int32_t* iters_out) {
  hipStream_t st = c->stream;
  const int nk = c->nk, npwx = c->npwx;
  const long nsys = (long)nk * nrhs;
  c->last_iterations = c->last_hpsi_kbands = c->last_graph_replays = 0;
  const size_t nv = (size_t)nsys * npwx;
  DevBufs bf(c);
  cd *r, *d, *dold, *t, *W;
  double *eps, *alpha, *rho, *rho_old, *tk;
  int* active;
  MKPW_TRY(bf.get(nv, &r));
  MKPW_TRY(bf.get(nv, &d));
  MKPW_TRY(bf.get(nv, &dold));
  MKPW_TRY(bf.get(nv, &t));
  MKPW_TRY(bf.get((size_t)nk * nocc * nrhs, &W));
  MKPW_TRY(bf.get((size_t)nsys, &eps));
  MKPW_TRY(bf.get((size_t)nk, &alpha));
  MKPW_TRY(bf.get((size_t)nsys, &rho));
  MKPW_TRY(bf.get((size_t)nsys, &rho_old));
  double* rho0;
  MKPW_TRY(bf.get((size_t)nsys, &rho0));
  MKPW_TRY(bf.get((size_t)nsys, &tk));
  MKPW_TRY(bf.get((size_t)nsys, &active));
  cplx<float>*v32 = nullptr, *t32 = nullptr;
  if (prec == PW_MIXED) {
    MKPW_TRY(bf.get(nv, &v32));
    MKPW_TRY(bf.get(nv, &t32));
  }
  MKPW_HIP(c, hipMemcpyAsync(eps, eps_h, sizeof(double) * nsys, hipMemcpyHostToDevice, st));
  MKPW_HIP(c, hipMemcpyAsync(alpha, alpha_h, sizeof(double) * nk, hipMemcpyHostToDevice, st));
  MKPW_HIP(c, hipMemsetAsync(dold, 0, sizeof(cd) * nv, st));
  MKPW_HIP(c, hipMemsetAsync(rho_old, 0, sizeof(double) * nsys, st));
  hipLaunchKernelGGL(tkin_kernel, dim3(nrhs, nk), dim3(256), 0, st, U, nocc, c->d_kin, c->d_npw, npwx, nrhs, tk);
  MKPW_TRY(check_launch(c, "tkin", st));
  // P = S U for the projector term (U itself without an overlap)
  const bool gen = c->have_q;
  const cd* P = U;
  if (gen) {
    cd* SU;
    MKPW_TRY(bf.get((size_t)nk * nocc * npwx, &SU));
    VecSel sel;
    sel.nvec = nocc;
    sel.kstride = (long)nocc * npwx;
    MKPW_TRY(launch_spsi(c, PW_FP64, sel, U, SU, nullptr, 0.0, st));
    P = SU;
  }

  bool fp64_h = prec == PW_FP64;
  // t = H v + alpha U (U^H v) for all systems
  // t = A v; with `live`, A is applied to the active systems only (the others'
  // t is not read)
  auto apply_a = [&](const cd* v, const int* live) -> pw_status {
    VecSel sel;
    sel.nvec = nrhs;
    sel.kstride = (long)nrhs * npwx;
    sel.live = live;
    if (fp64_h) {
      MKPW_TRY(launch_hpsi(c, PW_FP64, sel, v, t, st));
    } else {
      MKPW_TRY(
          launch_to_c64(c, v, (long)nrhs * npwx, nullptr, v32, (long)nrhs * npwx, nullptr, nullptr, nrhs, st, live));
      MKPW_TRY(launch_hpsi(c, PW_MIXED, sel, v32, t32, st));
      MKPW_TRY(
          launch_to_c128(c, t32, (long)nrhs * npwx, nullptr, t, (long)nrhs * npwx, nullptr, nullptr, nrhs, st, live));
    }
    if (gen) MKPW_TRY(launch_spsi(c, PW_FP64, sel, v, t, eps, -1.0, st));  // t -= eps S v
    GramArgs g;
    g.A = P; g.a_kstride = (long)nocc * npwx; g.a_n = nocc;
    g.B = v; g.b_kstride = (long)nrhs * npwx; g.b_n = nrhs;
    g.ld = npwx; g.npw = c->d_npw;
    g.C = W; g.c_kstride = (long)nocc * nrhs; g.ldc = nrhs;
    g.b_live = live; g.live_kstride = nrhs;
    MKPW_TRY(launch_gram(c, g, nocc, nrhs, st));
    hipLaunchKernelGGL(scale_w_kernel, dim3(nk), dim3(256), 0, st, W, nocc * nrhs, alpha);
    MKPW_TRY(check_launch(c, "scale_w", st));
    if (nocc > 64) return set_err(c, PW_EINVAL, "nocc must be <= 64");
    CombArgs m;
    m.X = P; m.x_kstride = (long)nocc * npwx; m.x_n = nocc;
    m.Y = t; m.y_kstride = (long)nrhs * npwx; m.y_n = nrhs;
    m.ld = npwx; m.Cm = W; m.c_kstride = (long)nocc * nrhs; m.ldc = nrhs;
    m.accumulate = 1;
    m.y_live = live; m.live_kstride = nrhs;
    MKPW_TRY(launch_combine(c, m, nocc, st));
    return PW_OK;
  };
  auto restart = [&]() -> pw_status {
    MKPW_TRY(apply_a(x, nullptr));
    hipLaunchKernelGGL(init_resid_kernel, dim3((unsigned)nsys), dim3(256), 0, st, t, x, b, eps, r, npwx, active,
                       c->d_npw, nrhs, gen ? 0 : 1);
    return check_launch(c, "init_resid", st);
  };

  // One unit of work is an update and the next check: t = A d on the active
  // systems, step 2 (x, r), step 1 (the next d, rho, convergence).  The host
  // reads only the number of systems still active, one unit late: the count
  // is copied to page-locked memory behind each unit and looked at once the
  // next unit is queued, so the device never waits for the host.  A unit
  // queued after every system has converged changes nothing (both step
  // kernels skip inactive systems, and t is scratch).  From the second unit of
  // a phase on, the unit runs as a captured graph, replayed.
  int* iters_d;
  int* d_nact;
  MKPW_TRY(bf.get((size_t)nsys, &iters_d));
  MKPW_TRY(bf.get((size_t)1, &d_nact));
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)std::min<long>(1024, (nsys + 255) / 256)), dim3(256), 0, st,
                     iters_d, nsys, 0);
  MKPW_TRY(check_launch(c, "fill", st));
  HostStage hs(c, st);
  MKPW_TRY(hs.init(0, 256 + sizeof(int) * nsys));
  int* slot[2] = {hs.back<int>(0), hs.back<int>(sizeof(int))};
  int* p_iters = hs.back<int>(256);
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct Cleanup {
    hipEvent_t* e;
    hipGraph_t* g;
    hipGraphExec_t* x;
    ~Cleanup() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
      if (*x) (void)hipGraphExecDestroy(*x);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } cleanup{ev, &graph, &exec};
  for (int i = 0; i < 2; ++i) MKPW_HIP(c, hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  auto drop_graph = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };

  auto step1 = [&](int first) -> pw_status {
    // the FP32 phase of the mixed mode stops at a residual reduction its
    // H application can still resolve; the FP64 phase runs to thr
    // rho reduction (squared M^-1-norm of the residual) at which the mixed
    // mode leaves complex64 H: by default 1e-10, a residual norm 1e-5 of the
    // starting one, near what an H application with FP32 rounding resolves
    const double rel = fp64_h ? 0.0 : std::pow(10.0, -(double)c->cg_switch_digits);
    hipLaunchKernelGGL(step1_kernel, dim3((unsigned)nsys), dim3(256), 0, st, r, d, dold, c->d_kin, tk, c->d_npw, npwx,
                       nrhs, rho, rho_old, rho0, active, first, thr, rel, iters_d);
    MKPW_TRY(check_launch(c, "cg_step1", st));
    hipLaunchKernelGGL(count_active_kernel, dim3(1), dim3(1024), 0, st, active, nsys, d_nact);
    return check_launch(c, "count_active", st);
  };
  auto unit = [&]() -> pw_status {
    MKPW_TRY(apply_a(d, active));
    hipLaunchKernelGGL(step2_kernel, dim3((unsigned)nsys), dim3(256), 0, st, t, d, dold, x, r, eps, c->d_npw, npwx,
                       nrhs, rho, rho_old, active, gen ? 0 : 1);
    MKPW_TRY(check_launch(c, "cg_step2", st));
    return step1(0);
  };
  bool use_graph = c->solver_graph && !c->trace;
  auto run_unit = [&](int in_phase) -> pw_status {
    if (use_graph && in_phase >= 2) {
      if (!exec) {
        bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
          pw_status s = unit();
          hipGraph_t g = nullptr;
          const bool ended = hipStreamEndCapture(st, &g) == hipSuccess;
          if (s != PW_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
          }
          ok = ended && g && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
          graph = g;
        }
        if (!ok) {  // run this and every later unit launch by launch
          (void)hipGetLastError();
          drop_graph();
          use_graph = false;
          return unit();
        }
      }
      MKPW_HIP(c, hipGraphLaunch(exec, st));
      ++c->last_graph_replays;
      return PW_OK;
    }
    return unit();
  };
  auto post = [&](int u) -> pw_status {
    MKPW_HIP(c, hipMemcpyAsync(slot[u & 1], d_nact, sizeof(int), hipMemcpyDeviceToHost, st));
    MKPW_HIP(c, hipEventRecord(ev[u & 1], st));
    return PW_OK;
  };

  MKPW_TRY(restart());
  c->last_hpsi_kbands += nsys;
  MKPW_TRY(step1(1));
  MKPW_TRY(post(0));
  bool ok = false;
  int phase_first = 1;  // first unit of the current phase
  int u = 1;
  for (u = 1;; ++u) {
    if (u <= max_iter) {
      MKPW_TRY(run_unit(u - phase_first + 1));
      MKPW_TRY(post(u));
    }
    // the check that preceded unit u
    MKPW_HIP(c, hipEventSynchronize(ev[(u - 1) & 1]));
    const int n_act = *slot[(u - 1) & 1];
    if (u <= max_iter) c->last_hpsi_kbands += n_act;
    if (n_act == 0) {
      if (!fp64_h) {
        // FP64 refinement: true residual with H in FP64, then continue
        fp64_h = true;
        drop_graph();
        MKPW_TRY(restart());
        c->last_hpsi_kbands += nsys;
        MKPW_TRY(step1(1));
        MKPW_TRY(post(u));
        phase_first = u + 1;
        continue;
      }
      ok = true;
      break;
    }
    if (u > max_iter) break;
  }
  c->last_iterations = std::min(u, max_iter);
  MKPW_HIP(c, hipMemcpyAsync(p_iters, iters_d, sizeof(int) * nsys, hipMemcpyDeviceToHost, st));
  MKPW_HIP(c, hipStreamSynchronize(st));
  if (iters_out)
    for (long s = 0; s < nsys; ++s) iters_out[s] = p_iters[s];
  if (!ok) return set_err(c, PW_ENOCONV, "CG: some systems did not converge");
  return PW_OK;
}

}  // namespace mkpw

extern "C" pw_status pw_dfpt_cg(pw_ctx* c, pw_prec prec, int nocc, const void* psi_occ, const double* eps_ha,
                                const double* alpha_ha, int nrhs, const void* rhs, void* dpsi, double thr,
                                int max_iter, int32_t* iters) {
  using namespace mkpw;
  if (!c) return PW_EINVAL;
  if (c->host_only) return set_err(c, PW_ESTATE, "host-only context runs no device work");
  if (!c->have_k || !c->have_v) return set_err(c, PW_ESTATE, "set k-points and potential before dfpt_cg");
  if (prec != PW_FP64 && prec != PW_MIXED) return set_err(c, PW_EINVAL, "unknown precision");
  if (!psi_occ || !eps_ha || !alpha_ha || !rhs || !dpsi) return set_err(c, PW_EINVAL, "null argument");
  if (nocc < 1 || nocc > 64) return set_err(c, PW_EINVAL, "nocc must be in [1, 64]");
  if (nrhs < 1 || nrhs > nocc) return set_err(c, PW_EINVAL, "nrhs must be in [1, nocc]");
  if (!(thr > 0.0)) return set_err(c, PW_EINVAL, "thr must be positive");
  if (max_iter < 1) return set_err(c, PW_EINVAL, "max_iter must be >= 1");
  for (int k = 0; k < c->nk; ++k)
    if (!(alpha_ha[k] > 0.0)) return set_err(c, PW_EINVAL, "alpha must be positive");
  (void)hipSetDevice(c->device);
  return dfpt_cg_run(c, prec, nocc, (const cplx<double>*)psi_occ, eps_ha, alpha_ha, nrhs, (const cplx<double>*)rhs,
                     (cplx<double>*)dpsi, thr, max_iter, iters);
}
