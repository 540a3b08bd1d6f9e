// Preconditioned conjugate gradients (section 2.3: CG applied to P K u = P f, Eq. eq-pre).
//
// FP64 throughout: residual, search direction, dot products and alpha / beta.  Dot
// products are two-pass deterministic reductions (per-block partials, then one block sums
// them in a fixed order); alpha and beta are formed on the device, so the host reads one
// scalar pair per iteration for the stopping test ||r|| <= rtol ||b||.
#include <cmath>
#include <memory>

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
  // split: the subdomain solves are left to the caller (a multi-set launch), which then
  // calls pcg_next_post; post_pending / post_first record that such a step is open
  bool split = false, post_pending = false, post_first = false;
  gx_status st = GX_OK;
  std::string msg;
  EventPair ev_spmv, ev_pre;
  double t_spmv = 0.0, t_pre = 0.0;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  hipEvent_t ready = nullptr;                      // local right-hand sides formed (split)
  ~PcgRun() {
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (ready) (void)hipEventDestroy(ready);
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

// after the subdomain solves: the rest of the preconditioner, beta, new direction, then
// the next body
static void pcg_next_post(PcgRun& R, bool first) {
  gx_ctx* c = R.c;
  hipStream_t s = c->stream;
  const int64_t n = 3 * c->n_nodes;
  R.post_pending = false;
  precond_finish(c, c->r.p, c->z.p);
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

// precond (local right-hand sides, subdomain solves unless split), then pcg_next_post
static void pcg_next(PcgRun& R, bool first) {
  gx_ctx* c = R.c;
  GX_HIP(hipEventRecord(R.ev_pre.a, c->stream));
  precond_local(c, c->r.p);
  if (R.split) {
    R.post_pending = true;
    R.post_first = first;
    return;
  }
  band_solve(c->sw.A, c->sw.d_xoff.p, c->sw.wr64.p, c->stream);
  pcg_next_post(R, first);
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
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return GX_EINVAL;
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) return GX_EINVAL;    // one system per context
  }
  std::vector<PcgRun> runs(n);
  std::vector<gx_status> st(n, GX_OK);
  auto fail = [&](int i, gx_status code, const char* what) {
    if (st[i] == GX_OK) st[i] = code;
    ctxs[i]->err = what;
    runs[i].done = true;
    runs[i].post_pending = false;
  };
  // the coarse solves of all systems run concurrently: each context's gets an equal share of
  // the machine (work-group counts chosen again), restored afterwards
  auto set_share = [&](int share) {
    for (int i = 0; i < n; ++i) {
      BandSet& bs = ctxs[i]->sw.C;
      bs.share = share;
      bs.solve_groups[0] = bs.solve_groups[1] = 0;
    }
  };
  set_share(n);
  for (int i = 0; i < n; ++i) {
    runs[i].c = ctxs[i];
    runs[i].b = b[i];
    runs[i].x = x[i];
    runs[i].rtol = rtol;
    runs[i].maxit = maxit;
    runs[i].split = true;
    try {
      ctxs[i]->err.clear();
      GX_HIP(hipSetDevice(ctxs[i]->device));
      GX_HIP(hipEventCreateWithFlags(&runs[i].ready, hipEventDisableTiming));
      pcg_begin(runs[i]);
    } catch (const Error& e) {
      fail(i, e.code, e.what());
    }
  }
  // The subdomain solves of every system that goes on, one launch per device and factor
  // precision.  The launches of a device go one after another on a stream of their own,
  // which waits for the systems' local right-hand sides; every system's stream then waits
  // for all of them, so each launch has the device to itself (the waits between its
  // work-groups need them all resident).  A table is planned again when its set of systems
  // changes.
  struct Lane {
    int dev = 0;
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
  };
  struct Joint {
    int dev = 0;
    bool fp32 = false;
    std::vector<int> members;
    MultiSolve ms;
  };
  std::vector<Lane> lanes;
  std::vector<std::unique_ptr<Joint>> joints;
  std::vector<char> joined(n, 0);
  auto lane_of = [&](int dev) -> Lane& {
    for (Lane& l : lanes)
      if (l.dev == dev) return l;
    Lane l;
    l.dev = dev;
    GX_HIP(hipSetDevice(dev));
    GX_HIP(hipStreamCreateWithFlags(&l.st, hipStreamNonBlocking));
    if (hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(l.st);
      throw Error(GX_EHIP, "hipEventCreateWithFlags failed");
    }
    lanes.push_back(l);
    return lanes.back();
  };
  auto joint_solves = [&](const std::vector<int>& cont) {
    for (auto& j : joints) j->members.clear();
    std::vector<Joint*> used;
    for (int i : cont) {
      const int dev = ctxs[i]->device;
      const bool f32 = ctxs[i]->sw.A.fp32;
      Joint* J = nullptr;
      for (auto& j : joints)
        if (j->dev == dev && j->fp32 == f32) J = j.get();
      if (!J) {
        joints.push_back(std::make_unique<Joint>());
        J = joints.back().get();
        J->dev = dev;
        J->fp32 = f32;
      }
      if (J->members.empty()) used.push_back(J);
      J->members.push_back(i);
    }
    for (Joint* J : used) {
      try {
        GX_HIP(hipSetDevice(J->dev));
        hipStream_t ls = lane_of(J->dev).st;
        bool same = J->ms.sets.size() == J->members.size();
        for (size_t k = 0; same && k < J->members.size(); ++k)
          same = J->ms.sets[k] == &ctxs[J->members[k]]->sw.A;
        if (!same) {
          std::vector<BandSet*> sets;
          std::vector<double*> xs;
          std::vector<const int64_t*> xo;
          for (int i : J->members) {
            Schwarz& sw = ctxs[i]->sw;
            sets.push_back(&sw.A);
            xs.push_back(sw.wr64.p);
            xo.push_back(sw.xoff.data());
          }
          multi_solve_plan(J->ms, sets, xs, xo, ls);
        }
        for (int i : J->members) {
          GX_HIP(hipEventRecord(runs[i].ready, ctxs[i]->stream));
          GX_HIP(hipStreamWaitEvent(ls, runs[i].ready, 0));
          joined[i] = 1;
        }
        multi_solve(J->ms, ls);
      } catch (const Error& e) {
        for (int i : J->members) fail(i, e.code, e.what());
      }
    }
    for (Lane& l : lanes) {
      try {
        GX_HIP(hipSetDevice(l.dev));
        GX_HIP(hipEventRecord(l.done, l.st));
        for (int i : cont)
          if (!runs[i].done && ctxs[i]->device == l.dev)
            GX_HIP(hipStreamWaitEvent(ctxs[i]->stream, l.done, 0));
      } catch (const Error& e) {
        for (int i : cont)
          if (ctxs[i]->device == l.dev) fail(i, e.code, e.what());
      }
    }
  };
  // lockstep: one synchronisation of every active stream per iteration
  for (;;) {
    bool any = false;
    std::vector<int> cont;
    for (int i = 0; i < n; ++i) {
      if (runs[i].done) continue;
      any = true;
      try {
        GX_HIP(hipSetDevice(ctxs[i]->device));
        GX_HIP(hipStreamSynchronize(ctxs[i]->stream));
        pcg_advance(runs[i]);
        if (runs[i].post_pending) cont.push_back(i);
      } catch (const Error& e) {
        fail(i, e.code, e.what());
      }
    }
    if (!any) break;
    if (cont.empty()) continue;
    joint_solves(cont);
    for (int i : cont) {
      if (runs[i].done) continue;
      try {
        GX_HIP(hipSetDevice(ctxs[i]->device));
        pcg_next_post(runs[i], runs[i].post_first);
      } catch (const Error& e) {
        fail(i, e.code, e.what());
      }
    }
  }
  for (auto& J : joints) {
    try {
      GX_HIP(hipSetDevice(J->dev));
      hipStream_t ls = lane_of(J->dev).st;
      GX_HIP(hipStreamSynchronize(ls));
      multi_solve_check(J->ms, ls);
    } catch (const Error& e) {
      for (int i = 0; i < n; ++i)
        if (joined[i] && ctxs[i]->device == J->dev && ctxs[i]->sw.A.fp32 == J->fp32)
          fail(i, e.code, e.what());
    }
  }
  joints.clear();                                  // tables freed before their streams go
  for (Lane& l : lanes) {
    (void)hipSetDevice(l.dev);
    (void)hipEventDestroy(l.done);
    (void)hipStreamDestroy(l.st);
  }
  gx_status first = GX_OK;
  for (int i = 0; i < n; ++i) {
    try {
      if (runs[i].started) pcg_end(runs[i], iters_out ? iters_out + i : nullptr,
                                   relres_out ? relres_out + i : nullptr);
    } catch (const Error& e) {
      fail(i, e.code, e.what());
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
  GX_REQUIRE(reps >= 1 && which >= 0 && which <= 5, "bad kernel id or repetition count");
  if (which == 5) {                                // the interior factorisation, alone
    if (!c->setup_done) throw Error(GX_ESTATE, "preconditioner not set up");
    double tot = 0.0;
    for (int k = 0; k < reps; ++k) tot += interior_refactor_ms(c);
    if (avg_ms) *avg_ms = tot / reps;
    if (bytes) *bytes = c->sw.A.env_flops;
    return GX_OK;
  }
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

gx_status gx_band_stats(gx_ctx* c, double* out) {
  GX_API_BEGIN(c)
  if (!c->setup_done) throw Error(GX_ESTATE, "preconditioner not set up");
  GX_REQUIRE(out, "null output");
  const BandSet& A = c->sw.A;
  double env = 0.0;
  for (int64_t e : A.env) env += (double)e;
  out[0] = (double)A.total;
  out[1] = env;
  out[2] = A.env_flops;
  out[3] = (double)c->neumann_entries;
  out[4] = (double)c->neumann_envelope;
  out[5] = c->neumann_flops;
  out[6] = band_solve_bytes(A, 1, nullptr, false);
  out[7] = band_solve_bytes(A, 1, nullptr, true);
  GX_API_END(c)
}

}  // extern "C"
