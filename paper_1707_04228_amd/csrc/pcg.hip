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
  if (!c->setup_done) throw Error(GX_ESTATE, "gx_geneo_setup has not been called");
  GX_REQUIRE(b && x && rtol > 0 && maxit >= 0, "bad arguments");
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
  Timer tm(s);
  EventPair ev_spmv, ev_pre;
  double t_spmv = 0, t_pre = 0;
  const unsigned gb = nblocks(n, 256);
  zero(c->red, s);
  hipLaunchKernelGGL(k_zero_fixed, dim3(gb), dim3(256), 0, s, n, c->fixed.p, x);
  spmv(c, x, c->q.p);
  hipLaunchKernelGGL(k_residual0, dim3(gb), dim3(256), 0, s, n, c->fixed.p, b, c->q.p,
                     c->r.p, c->bm.p, x);
  dot(c, c->bm.p, c->bm.p, S_BB, 0);
  dot(c, c->r.p, c->r.p, S_RR, 0);
  double h[S_N];
  to_host(h, c->red.p, S_N, s);
  const double nb = std::sqrt(h[S_BB]);
  if (!(nb > 0)) {
    GX_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
    GX_HIP(hipStreamSynchronize(s));
    if (iters_out) *iters_out = 0;
    if (relres_out) *relres_out = 0.0;
    if (hist) hist[0] = 0.0;
    c->phase_ms[5] = tm.ms();
    return GX_OK;
  }
  double rel = std::sqrt(h[S_RR]) / nb;
  if (hist) hist[0] = rel;
  int it = 0;
  gx_status st = GX_OK;
  if (rel > rtol) {
    GX_HIP(hipEventRecord(ev_pre.a, s));
    precond_apply(c, c->r.p, c->z.p);
    GX_HIP(hipEventRecord(ev_pre.b, s));
    dot(c, c->r.p, c->z.p, S_RZ, 0);
    GX_HIP(hipMemcpyAsync(c->p.p, c->z.p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    st = GX_ENOCONV;
    while (it < maxit) {
      GX_HIP(hipEventRecord(ev_spmv.a, s));
      spmv(c, c->p.p, c->q.p);
      GX_HIP(hipEventRecord(ev_spmv.b, s));
      dot(c, c->p.p, c->q.p, S_PQ, 1);
      hipLaunchKernelGGL(k_update, dim3(RG), dim3(RB), 0, s, n, c->red.p, c->p.p, c->q.p, x,
                         c->r.p, c->red.p + S_N);
      hipLaunchKernelGGL(k_finish, dim3(1), dim3(RB), 0, s, c->red.p + S_N, c->red.p, S_RR,
                         0);
      GX_HIP(hipGetLastError());
      to_host(h, c->red.p, S_N, s);
      t_pre += ev_pre.ms();
      t_spmv += ev_spmv.ms();
      ++it;
      if (h[S_FLAG] != 0.0) {
        st = GX_EBREAKDOWN;
        c->err = "CG breakdown: p^T K p <= 0 or not finite";
        break;
      }
      rel = std::sqrt(h[S_RR]) / nb;
      if (hist) hist[it] = rel;
      if (!std::isfinite(rel)) {
        st = GX_EBREAKDOWN;
        c->err = "CG breakdown: residual not finite";
        break;
      }
      if (rel <= rtol) {
        st = GX_OK;
        break;
      }
      GX_HIP(hipEventRecord(ev_pre.a, s));
      precond_apply(c, c->r.p, c->z.p);
      GX_HIP(hipEventRecord(ev_pre.b, s));
      dot(c, c->r.p, c->z.p, S_RZNEW, 2);
      hipLaunchKernelGGL(k_newdir, dim3(gb), dim3(256), 0, s, n, c->red.p, c->z.p, c->p.p);
    }
    if (st == GX_ENOCONV) c->err = "maximum number of iterations reached";
  }
  GX_HIP(hipStreamSynchronize(s));
  band_solve_check(c->sw.A, s);
  band_solve_check(c->sw.C, s);
  if (iters_out) *iters_out = it;
  if (relres_out) *relres_out = rel;
  c->phase_ms[5] = tm.ms();
  c->phase_ms[6] = t_pre;
  c->phase_ms[7] = t_spmv;
  c->pcg_iters = it;
  return st;
  GX_API_END(c)
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
