// Preconditioned conjugate gradients (section 2.3: CG applied to P K u = P f, Eq. eq-pre).
//
// FP64 throughout: residual, search direction, dot products and alpha / beta.  Dot
// products are two-pass deterministic reductions (per-block partials, then one block sums
// them in a fixed order); alpha and beta are formed on the device, so the host reads one
// scalar pair per iteration for the stopping test ||r|| <= rtol ||b||.
#include <cmath>

#include "gx_internal.h"

namespace gx {

constexpr int RB = 256;          // reduction block
constexpr int RG = 1024;         // reduction grid (partials)

enum { S_RZ = 0, S_PQ, S_ALPHA, S_RR, S_RZNEW, S_BETA, S_BB, S_FLAG, S_N };

__device__ inline double block_sum(double s, double* red) {
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;                                     // valid in thread 0
}

__global__ void __launch_bounds__(RB) k_dot(int64_t n, const double* a, const double* b,
                                            double* part) {
  __shared__ double red[RB / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)RG * RB)
    s += a[i] * b[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// mode 0: S[dst] = sum; 1: alpha = RZ / sum (PQ); 2: beta = sum / RZ, RZ = sum
__global__ void __launch_bounds__(RB) k_finish(const double* part, double* S, int dst,
                                               int mode) {
  __shared__ double red[RB / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < RG; i += RB) s += part[i];   // fixed order per thread
  s = block_sum(s, red);
  if (threadIdx.x != 0) return;
  S[dst] = s;
  if (mode == 1) {
    if (!(s > 0.0) || !isfinite(s)) S[S_FLAG] = 1.0;
    S[S_ALPHA] = S[S_RZ] / s;
  } else if (mode == 2) {
    S[S_BETA] = s / S[S_RZ];
    S[S_RZ] = s;
  }
}

// x += alpha p; r -= alpha q; partial ||r||^2
__global__ void __launch_bounds__(RB) k_update(int64_t n, const double* S, const double* p,
                                               const double* q, double* x, double* r,
                                               double* part) {
  __shared__ double red[RB / 64];
  const double al = S[S_ALPHA];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += (int64_t)RG * RB) {
    x[i] += al * p[i];
    const double ri = r[i] - al * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_newdir(int64_t n, const double* S, const double* z, double* p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + S[S_BETA] * p[i];
}

// r = b - q on free DOFs (0 on clamped), x = 0 on clamped
__global__ void k_residual0(int64_t n, const uint8_t* fixed, const double* b,
                            const double* q, double* r, double* bm, double* x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool f = fixed[i];
  bm[i] = f ? 0.0 : b[i];
  r[i] = f ? 0.0 : b[i] - q[i];
}
__global__ void k_zero_fixed(int64_t n, const uint8_t* fixed, double* x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && fixed[i]) x[i] = 0.0;
}

__global__ void k_fill_ones(int64_t n, const uint8_t* fixed, double* x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = fixed[i] ? 0.0 : 1.0 + 1e-3 * (double)(i % 7);
}

static void dot(gx_ctx* c, const double* a, const double* b, int dst, int mode) {
  const int64_t n = 3 * c->n_nodes;
  hipLaunchKernelGGL(k_dot, dim3(RG), dim3(RB), 0, c->stream, n, a, b, c->red.p + S_N);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, c->stream, c->red.p + S_N, c->red.p,
                     dst, mode);
}


// One PCG solve as a state machine: begin() enqueues the initial residual, advance() reads
// the scalars copied to the host at the previous step and enqueues the next iteration (or
// finishes).  Between the two the caller synchronises the context's stream, so that a
// batch of solves on several streams waits once per iteration for all of them.
struct PcgRun {
  gx_ctx* c = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  double rtol = 0.0;
  int maxit = 0;
  double* hist = nullptr;
  double nb = 0.0, rel = 0.0;
  int it = 0;
  bool started = false, done = false, init_pending = true;
  gx_status st = GX_OK;
  std::string msg;
  EventPair ev_spmv, ev_pre;
  double t_spmv = 0.0, t_pre = 0.0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  ~PcgRun() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
  }
};

static void pcg_copy_scalars(gx_ctx* c) {
  GX_HIP(hipMemcpyAsync(c->hred.p, c->red.p, S_N * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream));
}

// spmv, alpha, x and r updates, ||r||; then the scalars to the host
static void pcg_body(PcgRun& R) {
  gx_ctx* c = R.c;
  hipStream_t s = c->stream;
  const int64_t n = 3 * c->n_nodes;
  GX_HIP(hipEventRecord(R.ev_spmv.a, s));
  spmv(c, c->p.p, c->q.p);
  GX_HIP(hipEventRecord(R.ev_spmv.b, s));
  dot(c, c->p.p, c->q.p, S_PQ, 1);
  hipLaunchKernelGGL(k_update, dim3(RG), dim3(RB), 0, s, n, c->red.p, c->p.p, c->q.p, R.x,
                     c->r.p, c->red.p + S_N);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, s, c->red.p + S_N, c->red.p, S_RR, 0);
  GX_HIP(hipGetLastError());
  pcg_copy_scalars(c);
}

static void pcg_begin(PcgRun& R) {
  gx_ctx* c = R.c;
  if (!c->setup_done) throw Error(GX_ESTATE, "gx_geneo_setup has not been called");
  GX_REQUIRE(R.b && R.x && R.rtol > 0 && R.maxit >= 0, "bad arguments");
  hipStream_t s = c->stream;
  const int64_t n = 3 * c->n_nodes;
  if (c->r.n != (size_t)n) {
    c->r.alloc(n);
    c->z.alloc(n);
    c->p.alloc(n);
    c->q.alloc(n);
    c->bm.alloc(n);
    c->red.alloc(S_N + RG);
  }
  c->hred.alloc(S_N);
  GX_HIP(hipEventCreate(&R.t0));
  GX_HIP(hipEventCreate(&R.t1));
  GX_HIP(hipEventRecord(R.t0, s));
  const unsigned gb = nblocks(n, 256);
  zero(c->red, s);
  hipLaunchKernelGGL(k_zero_fixed, dim3(gb), dim3(256), 0, s, n, c->fixed.p, R.x);
  spmv(c, R.x, c->q.p);
  hipLaunchKernelGGL(k_residual0, dim3(gb), dim3(256), 0, s, n, c->fixed.p, R.b, c->q.p,
                     c->r.p, c->bm.p, R.x);
  dot(c, c->bm.p, c->bm.p, S_BB, 0);
  dot(c, c->r.p, c->r.p, S_RR, 0);
  pcg_copy_scalars(c);
  R.started = true;
}

// precond, beta, new direction, then the next body
static void pcg_next(PcgRun& R, bool first) {
  gx_ctx* c = R.c;
  hipStream_t s = c->stream;
  const int64_t n = 3 * c->n_nodes;
  GX_HIP(hipEventRecord(R.ev_pre.a, s));
  precond_apply(c, c->r.p, c->z.p);
  GX_HIP(hipEventRecord(R.ev_pre.b, s));
  if (first) {
    dot(c, c->r.p, c->z.p, S_RZ, 0);
    GX_HIP(hipMemcpyAsync(c->p.p, c->z.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    dot(c, c->r.p, c->z.p, S_RZNEW, 2);
    hipLaunchKernelGGL(k_newdir, dim3(nblocks(n, 256)), dim3(256), 0, s, n, c->red.p, c->z.p,
                       c->p.p);
  }
  pcg_body(R);
}

// the scalars of the last step are on the host (the stream has been synchronised)
static void pcg_advance(PcgRun& R) {
  gx_ctx* c = R.c;
  const double* h = c->hred.p;
  if (R.init_pending) {
    R.init_pending = false;
    R.nb = std::sqrt(h[S_BB]);
    if (!(R.nb > 0)) {                             // b = 0: x = 0
      GX_HIP(hipMemsetAsync(R.x, 0, 3 * c->n_nodes * sizeof(double), c->stream));
      R.rel = 0.0;
      if (R.hist) R.hist[0] = 0.0;
      R.done = true;
      return;
    }
    R.rel = std::sqrt(h[S_RR]) / R.nb;
    if (R.hist) R.hist[0] = R.rel;
    if (R.rel <= R.rtol) {
      R.done = true;
      return;
    }
    R.st = GX_ENOCONV;
    if (R.maxit == 0) {
      R.msg = "maximum number of iterations reached";
      R.done = true;
      return;
    }
    pcg_next(R, true);
    return;
  }
  R.t_pre += R.ev_pre.ms();
  R.t_spmv += R.ev_spmv.ms();
  ++R.it;
  if (h[S_FLAG] != 0.0) {
    R.st = GX_EBREAKDOWN;
    R.msg = "CG breakdown: p^T K p <= 0 or not finite";
    R.done = true;
    return;
  }
  R.rel = std::sqrt(h[S_RR]) / R.nb;
  if (R.hist) R.hist[R.it] = R.rel;
  if (!std::isfinite(R.rel)) {
    R.st = GX_EBREAKDOWN;
    R.msg = "CG breakdown: residual not finite";
    R.done = true;
    return;
  }
  if (R.rel <= R.rtol) {
    R.st = GX_OK;
    R.done = true;
    return;
  }
  if (R.it >= R.maxit) {
    R.msg = "maximum number of iterations reached";
    R.done = true;
    return;
  }
  pcg_next(R, false);
}

static void pcg_end(PcgRun& R, int32_t* iters_out, double* relres_out) {
  gx_ctx* c = R.c;
  GX_HIP(hipEventRecord(R.t1, c->stream));
  GX_HIP(hipStreamSynchronize(c->stream));
  band_solve_check(c->sw.A, c->stream);
  band_solve_check(c->sw.C, c->stream);
  if (iters_out) *iters_out = R.it;
  if (relres_out) *relres_out = R.rel;
  float ms = 0.0f;
  GX_HIP(hipEventElapsedTime(&ms, R.t0, R.t1));
  c->phase_ms[5] = ms;
  c->phase_ms[6] = R.t_pre;
  c->phase_ms[7] = R.t_spmv;
  c->pcg_iters = R.it;
  if (R.st != GX_OK) c->err = R.msg;
}

}  // namespace gx

using namespace gx;

extern "C" {

gx_status gx_precond_apply(gx_ctx* c, const double* r, double* z) {
  GX_API_BEGIN(c)
  if (!c->setup_done) throw Error(GX_ESTATE, "gx_geneo_setup has not been called");
  GX_REQUIRE(r && z && r != z, "bad vectors");
  precond_apply(c, r, z);
  GX_HIP(hipStreamSynchronize(c->stream));
  band_solve_check(c->sw.A, c->stream);
  band_solve_check(c->sw.C, c->stream);
  GX_API_END(c)
}

gx_status gx_pcg_solve(gx_ctx* c, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t* iters_out, double* relres_out, double* hist) {
  GX_API_BEGIN(c)
  PcgRun R;
  R.c = c;
  R.b = b;
  R.x = x;
  R.rtol = rtol;
  R.maxit = maxit;
  R.hist = hist;
  pcg_begin(R);
  while (!R.done) {
    GX_HIP(hipStreamSynchronize(c->stream));
    pcg_advance(R);
  }
  pcg_end(R, iters_out, relres_out);
  return R.st;
  GX_API_END(c)
}

gx_status gx_pcg_solve_batch(int32_t n, gx_ctx* const* ctxs, const double* const* b,
                             double* const* x, double rtol, int32_t maxit, int32_t* iters_out,
                             double* relres_out, int32_t* status_out) {
  if (n < 1 || !ctxs || !b || !x) return GX_EINVAL;
  std::vector<PcgRun> runs(n);
  std::vector<gx_status> st(n, GX_OK);
  auto fail = [&](int i, gx_status code, const char* what) {
    st[i] = code;
    ctxs[i]->err = what;
    runs[i].done = true;
  };
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return GX_EINVAL;
  // the solves of all systems run concurrently: each context's band solves get an equal
  // share of the machine (work-group counts chosen again), restored afterwards
  auto set_share = [&](int share) {
    for (int i = 0; i < n; ++i)
      for (BandSet* bs : {&ctxs[i]->sw.A, &ctxs[i]->sw.C}) {
        bs->share = share;
        bs->solve_groups[0] = bs->solve_groups[1] = 0;
      }
  };
  set_share(n);
  for (int i = 0; i < n; ++i) {
    runs[i].c = ctxs[i];
    runs[i].b = b[i];
    runs[i].x = x[i];
    runs[i].rtol = rtol;
    runs[i].maxit = maxit;
    try {
      ctxs[i]->err.clear();
      GX_HIP(hipSetDevice(ctxs[i]->device));
      pcg_begin(runs[i]);
    } catch (const Error& e) {
      fail(i, e.code, e.what());
    }
  }
  // lockstep: one synchronisation of every active stream per iteration
  for (;;) {
    bool any = false;
    for (int i = 0; i < n; ++i) {
      if (runs[i].done) continue;
      any = true;
      try {
        GX_HIP(hipSetDevice(ctxs[i]->device));
        GX_HIP(hipStreamSynchronize(ctxs[i]->stream));
        pcg_advance(runs[i]);
      } catch (const Error& e) {
        fail(i, e.code, e.what());
      }
    }
    if (!any) break;
  }
  gx_status first = GX_OK;
  for (int i = 0; i < n; ++i) {
    try {
      if (runs[i].started) pcg_end(runs[i], iters_out ? iters_out + i : nullptr,
                                   relres_out ? relres_out + i : nullptr);
    } catch (const Error& e) {
      if (st[i] == GX_OK) fail(i, e.code, e.what());
    }
    if (st[i] == GX_OK) st[i] = runs[i].st;
    if (status_out) status_out[i] = st[i];
    if (first == GX_OK) first = st[i];
  }
  set_share(1);
  return first;
}

gx_status gx_kernel_time(gx_ctx* c, int32_t which, int32_t reps, double* avg_ms,
                         double* bytes) {
  GX_API_BEGIN(c)
  GX_REQUIRE(reps >= 1 && which >= 0 && which <= 4, "bad kernel id or repetition count");
  if (which == 4) {                                // recorded during the last setup
    if (!c->setup_done || c->mrhs_calls == 0) throw Error(GX_ESTATE, "no eigensolver solves recorded");
    if (avg_ms) *avg_ms = c->mrhs_ms / (double)c->mrhs_calls;
    if (bytes) *bytes = c->mrhs_bytes / (double)c->mrhs_calls;
    return GX_OK;
  }
  if (!c->assembled) throw Error(GX_ESTATE, "matrix not assembled");
  if (which >= 1 && !c->setup_done) throw Error(GX_ESTATE, "preconditioner not set up");
  if (which == 3 && !(c->sw.two_level && c->sw.n0 > 0)) throw Error(GX_ESTATE, "no coarse space");
  hipStream_t s = c->stream;
  const int64_t n = 3 * c->n_nodes;
  if (c->r.n != (size_t)n) {
    c->r.alloc(n);
    c->z.alloc(n);
    c->p.alloc(n);
    c->q.alloc(n);
    c->bm.alloc(n);
    c->red.alloc(S_N + RG);
  }
  hipLaunchKernelGGL(k_fill_ones, dim3(nblocks(n, 256)), dim3(256), 0, s, n, c->fixed.p,
                     c->r.p);
  GX_HIP(hipMemcpyAsync(c->p.p, c->r.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  EventPair ev;
  double tot = 0.0, b = 0.0;
  Schwarz& sw = c->sw;
  for (int k = 0; k < reps; ++k) {
    if (which == 1) precond_apply(c, c->r.p, c->z.p);   // refills the local right-hand sides
    GX_HIP(hipEventRecord(ev.a, s));
    if (which == 0) spmv(c, c->p.p, c->q.p);
    if (which == 1) band_solve(sw.A, sw.d_xoff.p, sw.wr64.p, s);
    if (which == 2) precond_apply(c, c->r.p, c->z.p);
    if (which == 3) band_solve(sw.C, sw.d_c_xoff.p, sw.y0.p, s);
    GX_HIP(hipEventRecord(ev.b, s));
    GX_HIP(hipGetLastError());
    GX_HIP(hipEventSynchronize(ev.b));
    tot += ev.ms();
  }
  if (which == 0) b = (double)c->nnzb * (72 + 4) + (double)c->n_nodes * (4 + 24 + 24);
  if (which == 1 || which == 3) b = band_solve_bytes(which == 1 ? sw.A : sw.C, 1);
  if (avg_ms) *avg_ms = tot / reps;
  if (bytes) *bytes = b;
  GX_API_END(c)
}

}  // extern "C"
