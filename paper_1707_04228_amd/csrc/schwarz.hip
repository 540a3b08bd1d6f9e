// Overlapping decomposition and the additive two-level Schwarz preconditioner.
//
// Section 2.3 (Fig. fig-domaindecomp): subdomains of roughly equal size, grown by whole
// layers of elements, local problems with zero displacement on the artificial boundary
// solved exactly, local contributions glued by a partition of unity, plus a coarse
// correction (Eq. eq-pre):
//     z = P r = sum_j R_j^T A_j^-1 R_j r + Z K_0^-1 Z^T r.
//
// Subdomain membership is a bit mask per element and per node (64 subdomains per word):
// growth by node adjacency is two gathers per overlap layer, the interior nodes of
// subdomain j are the nodes all of whose elements carry bit j, and every per-subdomain
// node or element list comes out of one ballot-based stream compaction for all
// subdomains at once.
#include "gx_internal.h"

namespace gx {

// ---------------------------------------------------------------------------------------
// membership masks
__global__ void k_dd_init(const int32_t* part, int64_t E, int W, int n_sub, uint64_t* em,
                          int* err) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int p = part[e];
  if (p < 0 || p >= n_sub) {
    atomicOr(err, 1);
    return;
  }
  for (int w = 0; w < W; ++w) em[e * W + w] = (w == p / 64) ? (1ull << (p % 64)) : 0ull;
}

__global__ void k_dd_node(const int32_t* ne_ptr, const int32_t* ne_idx, const uint64_t* em,
                          int W, int64_t N, uint64_t* nor, uint64_t* nand) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int w = 0; w < W; ++w) {
    uint64_t o = 0, a = ~0ull;
    for (int k = ne_ptr[n]; k < ne_ptr[n + 1]; ++k) {
      const uint64_t m = em[(int64_t)ne_idx[k] * W + w];
      o |= m;
      a &= m;
    }
    nor[n * W + w] = o;
    if (nand) nand[n * W + w] = a;
  }
}

__global__ void k_dd_grow(const int32_t* conn, const uint64_t* nor, int W, int64_t E,
                          uint64_t* em) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  for (int w = 0; w < W; ++w) {
    uint64_t o = 0;
    for (int a = 0; a < 20; ++a) o |= nor[(int64_t)conn[20 * e + a] * W + w];
    em[e * W + w] = o;
  }
}

__global__ void k_node_count(const uint64_t* nand, int W, int64_t N, int32_t* cnt,
                             int* err) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int c = 0;
  for (int w = 0; w < W; ++w) c += __popcll(nand[n * W + w]);
  cnt[n] = c;
  if (c == 0) atomicOr(err, 1);
}

// ---------------------------------------------------------------------------------------
// ballot stream compaction of the items carrying bit j, for every j
constexpr int CH = 256;

__device__ inline uint64_t lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ void __launch_bounds__(CH) k_bits_count(const uint64_t* mask, int64_t n_items,
                                                   int W, int n_sub, int32_t* chunk_cnt) {
  extern __shared__ int32_t cnt[];
  for (int j = threadIdx.x; j < n_sub; j += CH) cnt[j] = 0;
  __syncthreads();
  const int64_t it = (int64_t)blockIdx.x * CH + threadIdx.x;
  const int lane = threadIdx.x & 63;
  for (int j = 0; j < n_sub; ++j) {
    const bool bit = it < n_items && ((mask[it * W + j / 64] >> (j % 64)) & 1ull);
    const uint64_t b = __ballot(bit);
    if (lane == 0 && b) atomicAdd(&cnt[j], __popcll(b));
  }
  __syncthreads();
  for (int j = threadIdx.x; j < n_sub; j += CH)
    chunk_cnt[(int64_t)blockIdx.x * n_sub + j] = cnt[j];
}

__global__ void k_chunk_scan(int32_t* chunk, int64_t n_chunks, int n_sub, int64_t* totals) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_sub) return;
  int64_t run = 0;
  for (int64_t c = 0; c < n_chunks; ++c) {
    const int32_t v = chunk[c * n_sub + j];
    chunk[c * n_sub + j] = (int32_t)run;
    run += v;
  }
  totals[j] = run;
}

__global__ void __launch_bounds__(CH) k_bits_scatter(const uint64_t* mask, int64_t n_items,
                                                     int W, int n_sub, const int32_t* chunk,
                                                     const int64_t* list_off, int32_t* list,
                                                     int32_t* loc) {
  __shared__ int32_t wc[CH / 64];
  const int64_t it = (int64_t)blockIdx.x * CH + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < n_sub; ++j) {
    const bool bit = it < n_items && ((mask[it * W + j / 64] >> (j % 64)) & 1ull);
    const uint64_t b = __ballot(bit);
    if (lane == 0) wc[wave] = __popcll(b);
    __syncthreads();
    if (bit) {
      int before = 0;
      for (int w = 0; w < wave; ++w) before += wc[w];
      const int32_t rank =
          chunk[(int64_t)blockIdx.x * n_sub + j] + before + __popcll(b & lanemask_lt(lane));
      list[list_off[j] + rank] = (int32_t)it;
      if (loc) loc[(int64_t)j * n_items + it] = rank;
    }
    __syncthreads();
  }
}

// Per-subdomain sorted lists of the items (nodes or elements) whose mask carries bit j.
static void compact(gx_ctx* c, const uint64_t* mask, int64_t n_items, int W, int n_sub,
                    std::vector<int64_t>& cnt, std::vector<int64_t>& off,
                    DevBuf<int64_t>& d_off, DevBuf<int64_t>& d_cnt, DevBuf<int32_t>& list,
                    DevBuf<int32_t>* loc) {
  hipStream_t s = c->stream;
  const int64_t nch = (n_items + CH - 1) / CH;
  DevBuf<int32_t> chunk(nch * n_sub);
  DevBuf<int64_t> tot(n_sub);
  hipLaunchKernelGGL(k_bits_count, dim3((unsigned)nch), dim3(CH), n_sub * sizeof(int32_t), s,
                     mask, n_items, W, n_sub, chunk.p);
  hipLaunchKernelGGL(k_chunk_scan, dim3(nblocks(n_sub, 64)), dim3(64), 0, s, chunk.p, nch,
                     n_sub, tot.p);
  GX_HIP(hipGetLastError());
  cnt.resize(n_sub);
  off.resize(n_sub + 1);
  to_host(cnt.data(), tot.p, n_sub, s);
  off[0] = 0;
  for (int j = 0; j < n_sub; ++j) off[j + 1] = off[j] + cnt[j];
  GX_REQUIRE(off[n_sub] < ((int64_t)1 << 31), "subdomain lists too large");
  d_off.alloc(n_sub + 1);
  d_cnt.alloc(n_sub);
  to_dev(d_off.p, off.data(), n_sub + 1, s);
  to_dev(d_cnt.p, cnt.data(), n_sub, s);
  list.alloc(std::max<int64_t>(off[n_sub], 1));
  if (loc) {
    loc->alloc((size_t)n_sub * n_items);
    GX_HIP(hipMemsetAsync(loc->p, 0xff, loc->bytes(), s));
  }
  hipLaunchKernelGGL(k_bits_scatter, dim3((unsigned)nch), dim3(CH), 0, s, mask, n_items, W,
                     n_sub, chunk.p, d_off.p, list.p, loc ? loc->p : nullptr);
  GX_HIP(hipGetLastError());
  GX_HIP(hipStreamSynchronize(s));
}

void dd_build(gx_ctx* c, const int32_t* part, int n_sub, int overlap) {
  Schwarz& sw = c->sw;
  hipStream_t s = c->stream;
  const int64_t N = c->n_nodes, E = c->n_elems;
  const int W = (n_sub + 63) / 64;
  sw.n_sub = n_sub;
  sw.W = W;
  sw.elem_mask.alloc((size_t)E * W);
  sw.node_or.alloc((size_t)N * W);
  sw.node_and.alloc((size_t)N * W);
  DevBuf<int> err(1);
  zero(err, s);
  hipLaunchKernelGGL(k_dd_init, dim3(nblocks(E, 256)), dim3(256), 0, s, part, E, W, n_sub,
                     sw.elem_mask.p, err.p);
  for (int l = 0; l < overlap; ++l) {
    hipLaunchKernelGGL(k_dd_node, dim3(nblocks(N, 256)), dim3(256), 0, s, c->ne_ptr.p,
                       c->ne_idx.p, sw.elem_mask.p, W, N, sw.node_or.p, (uint64_t*)nullptr);
    hipLaunchKernelGGL(k_dd_grow, dim3(nblocks(E, 256)), dim3(256), 0, s, c->conn.p,
                       sw.node_or.p, W, E, sw.elem_mask.p);
  }
  hipLaunchKernelGGL(k_dd_node, dim3(nblocks(N, 256)), dim3(256), 0, s, c->ne_ptr.p,
                     c->ne_idx.p, sw.elem_mask.p, W, N, sw.node_or.p, sw.node_and.p);
  sw.node_cnt.alloc(N);
  hipLaunchKernelGGL(k_node_count, dim3(nblocks(N, 256)), dim3(256), 0, s, sw.node_and.p, W,
                     N, sw.node_cnt.p, err.p + 0);
  GX_HIP(hipGetLastError());
  int h = 0;
  to_host(&h, err.p, 1, s);
  GX_REQUIRE(!h, "partition index out of range, or a node lies in no subdomain interior "
                 "(overlap must be >= 1 and every subdomain non-empty)");
  compact(c, sw.node_and.p, N, W, n_sub, sw.nI, sw.offI, sw.d_offI, sw.d_nI, sw.I_nodes,
          &sw.I_loc);
  compact(c, sw.node_or.p, N, W, n_sub, sw.nD, sw.offD, sw.d_offD, sw.d_nD, sw.D_nodes,
          &sw.D_loc);
  compact(c, sw.elem_mask.p, E, W, n_sub, sw.nE, sw.offE, sw.d_offE, sw.d_nE, sw.E_list,
          nullptr);
  for (int j = 0; j < n_sub; ++j)
    GX_REQUIRE(sw.nI[j] > 0, "subdomain " + std::to_string(j) + " has no interior node");
}

// ---------------------------------------------------------------------------------------
// interior band matrices A_j = K[I_j, I_j]
// Per subdomain: the half bandwidth in nodes (max over the list of ln - first coupled local
// node) and the envelope of the DOF-level lower triangle: the three rows of node ln start at
// DOF 3 mn (mn its first coupled local node), so they hold 9 (ln - mn) + 6 entries up to
// and including their diagonals.  Integer sums: the result does not depend on the order.
__global__ void k_band_width(const int32_t* rp, const int32_t* col, const int32_t* list,
                             const int64_t* loff, const int64_t* lcnt, const int32_t* loc,
                             int64_t N, int32_t* bw, unsigned long long* env, int32_t* first) {
  const int j = blockIdx.y;
  const int64_t ln = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ln >= lcnt[j]) return;
  const int n = list[loff[j] + ln];
  const int32_t* lj = loc + (int64_t)j * N;
  int mn = (int)ln;
  for (int k = rp[n]; k < rp[n + 1]; ++k) {
    const int lm = lj[col[k]];
    if (lm >= 0 && lm < mn) mn = lm;
  }
  atomicMax(&bw[j], (int)ln - mn);
  atomicAdd(&env[j], (unsigned long long)(9 * ((int64_t)ln - mn) + 6));
  first[loff[j] + ln] = mn;
}

template <class T>
__global__ void __launch_bounds__(64) k_band_fill(const int32_t* rp, const int32_t* col,
                                                  const double* val, const double* dg,
                                                  const int32_t* list, const int64_t* loff,
                                                  const int64_t* lcnt, const int32_t* loc,
                                                  int64_t N, BandView bv, T* v) {
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= lcnt[j]) return;
  const int n = list[loff[j] + ln];
  const int32_t* lj = loc + (int64_t)j * N;
  const int64_t B = bv.B[j], ld = bv.ld[j];
  T* base = v + bv.off[j];
  for (int64_t i = threadIdx.x; i < 3 * ld; i += 64) base[3 * ln * ld + i] = (T)0;
  __syncthreads();
  for (int k = rp[n] + threadIdx.x; k < rp[n + 1]; k += 64) {
    const int m = col[k];
    const int lm = lj[m];
    if (lm < 0 || lm > ln) continue;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const int64_t r = 3 * ln + a, cc = 3 * (int64_t)lm + b;
        if (cc > r) continue;
        double x = val[(int64_t)k * 9 + 3 * a + b];
        if (dg) x /= sqrt(dg[3 * (int64_t)n + a] * dg[3 * (int64_t)m + b]);
        base[r * ld + (cc - r + B)] = (T)x;
      }
  }
}

__global__ void k_diag(const int32_t* rp, const int32_t* col, const double* val, int64_t N,
                       double* dg) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int k = rp[n]; k < rp[n + 1]; ++k)
    if (col[k] == n)
      for (int a = 0; a < 3; ++a) dg[3 * n + a] = val[(int64_t)k * 9 + 4 * a];
}

// Half bandwidth (in DOFs) of K restricted to each subdomain's node list, in list order.
std::vector<int64_t> list_bandwidth(gx_ctx* c, const int32_t* list, const int64_t* d_off,
                                    const int64_t* d_cnt, const int32_t* loc,
                                    const std::vector<int64_t>& cnt,
                                    std::vector<int64_t>* env_out,
                                    std::vector<int32_t>* first_out) {
  hipStream_t s = c->stream;
  const int n_sub = (int)cnt.size();
  int64_t mx = 0;
  for (int64_t v : cnt) mx = std::max(mx, v);
  std::vector<int64_t> hoff(n_sub + 1);
  to_host(hoff.data(), d_off, n_sub + 1, s);
  DevBuf<int32_t> bw(n_sub), first(std::max<int64_t>(hoff[n_sub], 1));
  DevBuf<unsigned long long> env(n_sub);
  zero(bw, s);
  zero(env, s);
  hipLaunchKernelGGL(k_band_width, dim3(nblocks(mx, 256), n_sub), dim3(256), 0, s,
                     c->row_ptr.p, c->col.p, list, d_off, d_cnt, loc, c->n_nodes, bw.p, env.p,
                     first.p);
  GX_HIP(hipGetLastError());
  if (first_out) {                                  // the matrices' nodes in order
    std::vector<int32_t> all(hoff[n_sub]);
    to_host(all.data(), first.p, all.size(), s);
    first_out->clear();
    for (int j = 0; j < n_sub; ++j)
      first_out->insert(first_out->end(), all.begin() + hoff[j], all.begin() + hoff[j] + cnt[j]);
  }
  std::vector<int32_t> hb(n_sub);
  std::vector<unsigned long long> he(n_sub);
  to_host(hb.data(), bw.p, n_sub, s);
  to_host(he.data(), env.p, n_sub, s);
  std::vector<int64_t> B(n_sub);
  for (int j = 0; j < n_sub; ++j) B[j] = 3 * (int64_t)hb[j] + 2;
  if (env_out) env_out->assign(he.begin(), he.end());
  return B;
}

// Fills the interior band matrices and enqueues their factorisation on s (which may be a
// side stream: nothing here waits for it); interior_factors_finish completes the job.
void interior_factors_prepare(gx_ctx* c, int precision, hipStream_t s, InteriorJob& job) {
  Schwarz& sw = c->sw;
  const int64_t N = c->n_nodes;
  const int n_sub = sw.n_sub;
  job.maxI = 0;
  for (int j = 0; j < n_sub; ++j) job.maxI = std::max(job.maxI, sw.nI[j]);
  job.B = list_bandwidth(c, sw.I_nodes.p, sw.d_offI.p, sw.d_nI.p, sw.I_loc.p, sw.nI, &job.env,
                         &job.first);
  job.n.assign(n_sub, 0);
  for (int j = 0; j < n_sub; ++j) job.n[j] = 3 * sw.nI[j];
  sw.precision = precision;
  job.fp32 = precision == GX_MIXED;
  band_layout(sw.A, job.n, job.B, job.fp32, s, &job.first);
  sw.A.force_groups[0] = c->tune[0];
  sw.A.force_groups[1] = c->tune[1];
  if (job.fp32) {
    sw.dg.alloc(3 * N);
    hipLaunchKernelGGL(k_diag, dim3(nblocks(N, 256)), dim3(256), 0, s, c->row_ptr.p,
                       c->col.p, c->val.p, N, sw.dg.p);
  }
  BandView bv{sw.A.d_B.p, sw.A.d_ld.p, sw.A.d_off.p};
  if (job.fp32)
    hipLaunchKernelGGL(k_band_fill<float>, dim3((unsigned)job.maxI, n_sub), dim3(64), 0, s,
                       c->row_ptr.p, c->col.p, c->val.p, sw.dg.p, sw.I_nodes.p, sw.d_offI.p,
                       sw.d_nI.p, sw.I_loc.p, N, bv, sw.A.v32.p);
  else
    hipLaunchKernelGGL(k_band_fill<double>, dim3((unsigned)job.maxI, n_sub), dim3(64), 0, s,
                       c->row_ptr.p, c->col.p, c->val.p, (const double*)nullptr, sw.I_nodes.p,
                       sw.d_offI.p, sw.d_nI.p, sw.I_loc.p, N, bv, sw.A.v64.p);
  GX_HIP(hipGetLastError());
}

void interior_factors_launch(gx_ctx* c, hipStream_t s, InteriorJob& job, bool threaded) {
  band_factor_start(c->sw.A, s, job.factor, "the subdomain matrices", threaded);
}

void interior_factors_start(gx_ctx* c, int precision, hipStream_t s, InteriorJob& job) {
  interior_factors_prepare(c, precision, s, job);
  interior_factors_launch(c, s, job, false);
}

// Waits for the factorisation (an FP32 breakdown is redone in FP64 on the context's
// stream, reported), then the solve work vectors, one segment of 3 nI_j per subdomain.
void interior_factors_finish(gx_ctx* c, InteriorJob& job) {
  Schwarz& sw = c->sw;
  hipStream_t s = c->stream;
  const int64_t N = c->n_nodes;
  const int n_sub = sw.n_sub;
  try {
    band_factor_finish(job.factor);
  } catch (const Error& e) {
    if (!job.fp32 || e.code != GX_ENOTSPD) throw;
    c->fp64_fallbacks |= 1;
    band_layout(sw.A, job.n, job.B, false, s, &job.first);
    BandView bv64{sw.A.d_B.p, sw.A.d_ld.p, sw.A.d_off.p};
    hipLaunchKernelGGL(k_band_fill<double>, dim3((unsigned)job.maxI, n_sub), dim3(64), 0, s,
                       c->row_ptr.p, c->col.p, c->val.p, (const double*)nullptr, sw.I_nodes.p,
                       sw.d_offI.p, sw.d_nI.p, sw.I_loc.p, N, bv64, sw.A.v64.p);
    GX_HIP(hipGetLastError());
    band_factor(sw.A, s, "the subdomain matrices");
    sw.precision = GX_FP64;
  }
  std::vector<int64_t> xo(n_sub + 1, 0);
  for (int j = 0; j < n_sub; ++j) xo[j + 1] = xo[j] + job.n[j];
  sw.xoff = xo;
  sw.d_xoff.alloc(n_sub + 1);
  to_dev(sw.d_xoff.p, xo.data(), n_sub + 1, s);
  sw.wr64.alloc(xo[n_sub]);                      // FP64 local vectors in both precisions
  GX_HIP(hipStreamSynchronize(s));
}

void interior_factors(gx_ctx* c, int precision) {
  InteriorJob job;
  interior_factors_start(c, precision, c->stream, job);
  interior_factors_finish(c, job);
}

// The interior band matrices filled again from K and factored once more, in the precision
// of the set-up, alone on the context's stream; returns the factorisation's duration (ms,
// HIP events around the factorisation kernels, the fill excluded).  The factors come out
// bit for bit as before (same kernels, same order).
double interior_refactor_ms(gx_ctx* c) {
  Schwarz& sw = c->sw;
  hipStream_t s = c->stream;
  const int64_t N = c->n_nodes;
  const int n_sub = sw.n_sub;
  int64_t maxI = 0;
  for (int j = 0; j < n_sub; ++j) maxI = std::max(maxI, sw.nI[j]);
  BandView bv{sw.A.d_B.p, sw.A.d_ld.p, sw.A.d_off.p};
  if (sw.A.fp32)
    hipLaunchKernelGGL(k_band_fill<float>, dim3((unsigned)maxI, n_sub), dim3(64), 0, s,
                       c->row_ptr.p, c->col.p, c->val.p, sw.dg.p, sw.I_nodes.p, sw.d_offI.p,
                       sw.d_nI.p, sw.I_loc.p, N, bv, sw.A.v32.p);
  else
    hipLaunchKernelGGL(k_band_fill<double>, dim3((unsigned)maxI, n_sub), dim3(64), 0, s,
                       c->row_ptr.p, c->col.p, c->val.p, (const double*)nullptr, sw.I_nodes.p,
                       sw.d_offI.p, sw.d_nI.p, sw.I_loc.p, N, bv, sw.A.v64.p);
  GX_HIP(hipGetLastError());
  EventPair ev;
  GX_HIP(hipEventRecord(ev.a, s));
  {
    FactorJob job;
    band_factor_start(sw.A, s, job, "the subdomain matrices");
    GX_HIP(hipEventRecord(ev.b, s));
    band_factor_finish(job);
  }
  GX_HIP(hipEventSynchronize(ev.b));
  return ev.ms();
}

// ---------------------------------------------------------------------------------------
// applying P
template <class V>
__global__ void k_gather_local(const double* r, const double* dg, const int32_t* list,
                               const int64_t* loff, const int64_t* lcnt, const int64_t* xoff,
                               V* w) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * lcnt[j]) return;
  const int64_t d = 3 * (int64_t)list[loff[j] + i / 3] + i % 3;
  double x = r[d];
  if (dg) x /= sqrt(dg[d]);
  w[xoff[j] + i] = (V)x;
}

// restriction Z_j^T r: partial sums over chunks of 1024 local rows
constexpr int RCH = 1024;
__global__ void __launch_bounds__(256) k_restrict(const double* r, const int32_t* list,
                                                  const int64_t* loff, const int64_t* lcnt,
                                                  const int64_t* zoff, const int32_t* nev,
                                                  const int32_t* coff, int64_t nchunk_max,
                                                  const double* Z, double* part) {
  __shared__ double red[4];
  const int j = blockIdx.y;
  const int64_t nj = 3 * lcnt[j];
  const int64_t r0 = (int64_t)blockIdx.x * RCH;
  const int m = nev[j];
  const double* Zj = Z + zoff[j];
  for (int a = 0; a < m; ++a) {
    double s = 0.0;
    if (r0 < nj)
      for (int64_t i = r0 + threadIdx.x; i < min(nj, r0 + RCH); i += 256)
        s += Zj[(int64_t)a * nj + i] * r[3 * (int64_t)list[loff[j] + i / 3] + i % 3];
    s = wave_sum_d(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
      part[(int64_t)(coff[j] + a) * nchunk_max + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

__global__ void k_restrict_sum(const double* part, int64_t n0, int64_t nchunk, double* y0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0) return;
  double s = 0.0;
  for (int64_t k = 0; k < nchunk; ++k) s += part[i * nchunk + k];
  y0[i] = s;
}

// z[d] = sum over subdomains j holding node(d) as interior of the local solution (and the
// coarse prolongation Z_j y_j); clamped DOFs stay zero
template <class V>
__global__ void k_combine(const uint64_t* nand, int W, int64_t N, const int32_t* I_loc,
                          const int64_t* xoff, const V* w, const double* dg,
                          const int64_t* zoff, const int32_t* nev, const int32_t* coff,
                          const int64_t* lcnt, const double* Z, const double* y0,
                          const uint8_t* fixed, double* z) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= 3 * N) return;
  const int64_t n = d / 3;
  const int comp = (int)(d % 3);
  double acc = 0.0, crs = 0.0;
  for (int wd = 0; wd < W; ++wd) {
    uint64_t bits = nand[n * W + wd];
    while (bits) {
      const int bpos = __ffsll((unsigned long long)bits) - 1;
      bits &= bits - 1;
      const int j = wd * 64 + bpos;
      const int64_t li = 3 * (int64_t)I_loc[(int64_t)j * N + n] + comp;
      acc += (double)w[xoff[j] + li];
      if (Z) {
        const int64_t nj = 3 * lcnt[j];
        const double* Zj = Z + zoff[j];
        const double* yj = y0 + coff[j];
        for (int a = 0; a < nev[j]; ++a) crs += Zj[(int64_t)a * nj + li] * yj[a];
      }
    }
  }
  if (dg) acc /= sqrt(dg[d]);                    // undo the symmetric scaling of A_j
  z[d] = fixed[d] ? 0.0 : acc + crs;
}

static int64_t max_interior(const Schwarz& sw) {
  int64_t maxI = 0;
  for (int j = 0; j < sw.n_sub; ++j) maxI = std::max(maxI, sw.nI[j]);
  return maxI;
}

// The local right-hand sides R_j r (scaled by the diagonal for FP32 factors).
void precond_local(gx_ctx* c, const double* r) {
  Schwarz& sw = c->sw;
  const int64_t maxI = max_interior(sw);
  const double* dg = sw.precision == GX_MIXED ? sw.dg.p : nullptr;
  hipLaunchKernelGGL(k_gather_local<double>, dim3(nblocks(3 * maxI, 256), sw.n_sub),
                     dim3(256), 0, c->stream, r, dg, sw.I_nodes.p, sw.d_offI.p, sw.d_nI.p,
                     sw.d_xoff.p, sw.wr64.p);
}

// After the local solves: the coarse correction and z = sum_j R_j^T D_j (local solution)
// plus the coarse part.
void precond_finish(gx_ctx* c, const double* r, double* z) {
  Schwarz& sw = c->sw;
  hipStream_t s = c->stream;
  const int64_t N = c->n_nodes;
  const int64_t maxI = max_interior(sw);
  const double* dg = sw.precision == GX_MIXED ? sw.dg.p : nullptr;
  const bool two = sw.two_level && sw.n0 > 0;
  if (two) {
    const int64_t nch = (3 * maxI + RCH - 1) / RCH;
    hipLaunchKernelGGL(k_restrict, dim3((unsigned)nch, sw.n_sub), dim3(256), 0, s, r,
                       sw.I_nodes.p, sw.d_offI.p, sw.d_nI.p, sw.d_z_off.p, sw.d_nev.p,
                       sw.d_c_off.p, nch, sw.Z.p, sw.y0part.p);
    hipLaunchKernelGGL(k_restrict_sum, dim3(nblocks(sw.n0, 256)), dim3(256), 0, s,
                       sw.y0part.p, sw.n0, nch, sw.y0.p);
    band_solve(sw.C, sw.d_c_xoff.p, sw.y0.p, s);
  }
  hipLaunchKernelGGL(k_combine<double>, dim3(nblocks(3 * N, 256)), dim3(256), 0, s,
                     sw.node_and.p, sw.W, N, sw.I_loc.p, sw.d_xoff.p, sw.wr64.p, dg,
                     sw.d_z_off.p, sw.d_nev.p, sw.d_c_off.p, sw.d_nI.p,
                     two ? sw.Z.p : nullptr, sw.y0.p, c->fixed.p, z);
  GX_HIP(hipGetLastError());
}

void precond_apply(gx_ctx* c, const double* r, double* z) {
  precond_local(c, r);
  band_solve(c->sw.A, c->sw.d_xoff.p, c->sw.wr64.p, c->stream);
  precond_finish(c, r, z);
}

}  // namespace gx
