// Batched banded Cholesky factorisation and triangular solves.
//
// The local problems of the overlapping Schwarz method are solved exactly by a direct
// method (section 2.4: sparse direct subdomain and coarse solves).  In the laminate DOF
// order (through-thickness planes outermost) every subdomain matrix is banded with a
// half bandwidth of about two lattice planes, so its Cholesky factor fits in band storage
// with no fill outside the band.
//
// Storage of matrix j: entry (r, c), r - B_j <= c <= r, at off_j + r * ld_j + (c - r + B_j).
//
// Factorisation: right-looking, block columns of NB; per step one kernel factors the
// diagonal block in LDS (and keeps its inverse for the solves), one solves the panel rows,
// one updates the trailing window with 64x64 tiles.  Matrices of different size and
// bandwidth run in the same launches.
//
// Solves: see the comment above the solve kernels.
#include <algorithm>

#include "gx_internal.h"

namespace gx {

constexpr int NB = 64;          // factorisation block
constexpr int TS = 64;          // trailing-update tile
constexpr int SB = 64;          // solve block (one wavefront)
constexpr int SOLVE_THREADS = 512;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// The 16x16x4 matrix instruction in the precision of a factor: FP64 factors multiply in FP64,
// FP32 factors (the mixed path) in FP32.  Both take A[l % 16][l / 16] and B[l / 16][l % 16]
// from lane l; the output row of accumulator register q differs: 4 q + l / 16 in FP64,
// 4 (l / 16) + q in FP32.  S is the type staged in LDS and multiplied.
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double S;
  typedef v4d V;
  static __device__ inline V mma(S a, S b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int q, int lk) { return 4 * q + lk; }
};
template <>
struct Mfma<float> {
  typedef float S;
  typedef v4f V;
  static __device__ inline V mma(S a, S b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int q, int lk) { return 4 * lk + q; }
};

struct BandArgs {
  const int64_t* n;
  const int64_t* B;
  const int64_t* ld;
  const int64_t* off;
};

// Diagonal block of step c0: Cholesky in LDS, written back; its inverse goes to inv[j].
template <class T>
__global__ void __launch_bounds__(256) k_potrf(BandArgs a, T* v, int64_t c0, double* inv,
                                               T* dinv, const int64_t* boff, int* err) {
  __shared__ double D[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  const int j = blockIdx.x;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (c0 >= n) return;
  T* base = v + a.off[j];
  const int nb = (int)min<int64_t>(NB, n - c0);
  {
    constexpr int L = NB * NB / 256;
    double vd[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int idx = threadIdx.x + 256 * u;
      const int i = idx / NB, l = idx % NB;
      double x = (i == l && i >= nb) ? 1.0 : 0.0;
      if (i < nb && l <= i && i - l <= B) x = (double)base[(c0 + i) * ld + (l - i + B)];
      vd[u] = x;
    }
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int idx = threadIdx.x + 256 * u;
      D[idx / NB][idx % NB] = vd[u];
    }
  }
  __syncthreads();
  // right-looking elimination on the unscaled columns: step i subtracts
  // D[r][i] D[s][i] / D[i][i] from the trailing lower triangle (s <= r); the columns are
  // scaled by 1/sqrt(pivot) at the end.  A non-positive pivot is reported and replaced by 1.
  // The steps go in blocks of BK columns, with the same operations in the same order per
  // entry: (1) wave 0 eliminates the BK x BK diagonal block in registers (lane r: row r,
  // pivots and column entries from wave-uniform lane reads), (2) one thread per row below
  // it applies the block's steps to its BK panel entries in registers and keeps the
  // multipliers f = D[r][i] / D[i][i], (3) all threads apply the block's steps to the
  // trailing lower triangle.  Three barriers per block instead of one per column.
  constexpr int BK = 16;
  __shared__ double piv[NB];
  __shared__ double F[NB][BK + 1];                 // multipliers of the current block
  {
    for (int k0 = 0; k0 < nb; k0 += BK) {
      const int kn = min(BK, nb - k0);             // steps of this block
      if (threadIdx.x < 64) {                      // (1) diagonal block
        const int lane = threadIdx.x;
        const int rr = min(lane, BK - 1);
        double a[BK];
#pragma unroll
        for (int c = 0; c < BK; ++c) a[c] = D[k0 + rr][k0 + c];
#pragma unroll
        for (int i = 0; i < BK; ++i) {
          if (i < kn) {
            const double dii = lane_value(a[i], i);
            const double d = dii > 0.0 ? dii : 1.0;
            const double f = a[i] / d;
#pragma unroll
            for (int s2 = i + 1; s2 < BK; ++s2) {
              const double dsi = lane_value(a[i], s2);      // D[k0 + s2][k0 + i]
              if (lane > i && lane < BK && s2 <= lane) a[s2] -= f * dsi;
            }
            if (lane == 0) {
              if (!(dii > 0.0)) atomicOr(err, 1);
              piv[k0 + i] = d;
            }
          }
        }
        if (lane < BK)
#pragma unroll
          for (int c = 0; c < BK; ++c)
            if (c <= lane) D[k0 + lane][k0 + c] = a[c];
      }
      __syncthreads();
      const int r0 = k0 + BK;                      // first row below the block
      if (r0 + (int)threadIdx.x < NB) {            // (2) panel rows
        const int r = r0 + threadIdx.x;
        double p[BK];
#pragma unroll
        for (int c = 0; c < BK; ++c) p[c] = D[r][k0 + c];
#pragma unroll
        for (int i = 0; i < BK; ++i) {
          if (i < kn) {
            const double f = p[i] / piv[k0 + i];
            F[r][i] = f;
#pragma unroll
            for (int s2 = i + 1; s2 < BK; ++s2) p[s2] -= f * D[k0 + s2][k0 + i];
          }
        }
#pragma unroll
        for (int c = 0; c < BK; ++c) D[r][k0 + c] = p[c];
      }
      __syncthreads();
      // (3) trailing lower triangle rows and columns r0 .. NB - 1, entry e -> (r, s)
      const int nt = NB - r0;
      for (int e = threadIdx.x; e < nt * (nt + 1) / 2; e += blockDim.x) {
        int r = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((r + 1) * (r + 2) / 2 <= e) ++r;
        while (r * (r + 1) / 2 > e) --r;
        const int s2 = e - r * (r + 1) / 2;
        double x = D[r0 + r][r0 + s2];
        for (int i = 0; i < kn; ++i) x -= F[r0 + r][i] * D[r0 + s2][k0 + i];
        D[r0 + r][r0 + s2] = x;
      }
      __syncthreads();
    }
    for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
      const int rr = idx / NB, c = idx % NB;
      if (c < nb && rr < nb && c <= rr) D[rr][c] = (rr == c) ? sqrt(piv[c]) : D[rr][c] / sqrt(piv[c]);
    }
    __syncthreads();
  }
  // inverse of the lower triangle (padding rows are identity): column c by forward
  // substitution, four threads per column (thread t: column t / 4, rows q = t mod 4 of
  // every four, kept in registers); each row's sum is combined across the four by two lane
  // exchanges
  if (threadIdx.x < NB) piv[threadIdx.x] = 1.0 / D[threadIdx.x][threadIdx.x];
  __syncthreads();
  {
    const int c = threadIdx.x >> 2, q = threadIdx.x & 3;
    double xr[NB / 4];
#pragma unroll
    for (int m = 0; m < NB / 4; ++m) xr[m] = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double part = 0.0;
#pragma unroll
      for (int m = 0; m < (i + 3) / 4; ++m)
        if (4 * m + q < i) part += D[i][4 * m + q] * xr[m];
      part += __shfl_xor(part, 1);
      part += __shfl_xor(part, 2);
      const double xi = ((i == c ? 1.0 : 0.0) - part) * piv[i];
      if (q == (i & 3)) xr[i >> 2] = xi;
    }
#pragma unroll
    for (int m = 0; m < NB / 4; ++m) Li[4 * m + q][c] = xr[m];
  }
  __syncthreads();
  double* ij = inv + (int64_t)j * NB * NB;
  T* dj = dinv + boff[j] + (c0 / NB) * NB * NB;   // kept for the triangular solves
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int i = idx / NB, l = idx % NB;
    ij[idx] = Li[i][l];
    dj[idx] = (T)Li[i][l];
    if (i < nb && l <= i && i - l <= B) base[(c0 + i) * ld + (l - i + B)] = (T)D[i][l];
  }
}

// panel rows r in [c0 + nb, c0 + nb + min(B, n - c0 - nb)): L[r, blk] = A[r, blk] L_kk^-T,
// 64 rows per work-group as a GEMM against the inverted diagonal block
template <class T>
__global__ void __launch_bounds__(256) k_trsm(BandArgs a, T* v, int64_t c0, const double* inv) {
  __shared__ double A[TS][NB + 1];
  __shared__ double Li[NB][NB + 1];
  const int j = blockIdx.y;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (c0 >= n) return;
  const int nb = (int)min<int64_t>(NB, n - c0);
  const int64_t nrow = min<int64_t>(B, n - c0 - nb);
  const int64_t r0 = c0 + nb + (int64_t)blockIdx.x * TS;
  if ((int64_t)blockIdx.x * TS >= nrow) return;
  T* base = v + a.off[j];
  const double* ij = inv + (int64_t)j * NB * NB;
  {
    constexpr int L = TS * NB / 256;             // 16 loads per thread, issued together
    double va[L], vl[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int idx = threadIdx.x + 256 * u;
      const int i = idx / NB, k = idx % NB;
      const int64_t r = r0 + i, col = c0 + k;
      va[u] = (k < nb && r - c0 - nb < nrow && col >= r - B) ? (double)base[r * ld + (col - r + B)]
                                                             : 0.0;
      vl[u] = ij[idx];
    }
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int idx = threadIdx.x + 256 * u;
      A[idx / NB][idx % NB] = va[u];
      Li[idx / NB][idx % NB] = vl[u];
    }
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int k = 0; k < NB; ++k) {
    double ar[4], lc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) ar[p] = A[4 * ty + p][k];
#pragma unroll
    for (int q = 0; q < 4; ++q) lc[q] = Li[4 * tx + q][k];      // X = A Li^T
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] += ar[p] * lc[q];
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t r = r0 + 4 * ty + p;
    if (r - c0 - nb >= nrow) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 4 * tx + q;
      const int64_t col = c0 + k;
      if (k < nb && col >= r - B) base[r * ld + (col - r + B)] = (T)acc[p][q];
    }
  }
}

// Update by the panels of columns [k0, k0 + kk): A[r][s] -= sum_c L[r][c] L[s][c] for
// t0 <= s <= r < t0 + W, t0 = k0 + kk, W = min(B, n - t0) (rows further down get nothing
// from these columns inside the band).  64x64 tiles of that lower triangle, or with
// col_only the first tile column only (the look-ahead update of the next panel inside a
// group).  The reduction runs over 64-column chunks of the panels: each chunk's two 64x64
// blocks are staged in LDS and each of the
// eight waves forms a 16x32 eighth of the tile with the FP64 matrix instruction (1x2 tiles
// of 16x16, 16 steps of k = 4); two work-groups fit a compute unit.  Lane l supplies row l % 16 and reduction index l / 16 of both
// operands; accumulator register q of a tile holds output row 4 q + l / 16, column l % 16.
// Grouping panels makes one read-modify-write pass over the trailing band serve kk columns.
constexpr int ST = 512;                           // threads of the trailing update

template <class T>
__global__ void __launch_bounds__(ST) k_syrk(BandArgs a, T* v, int64_t k0, int64_t kk,
                                             int col_only, int64_t ts_lo, int64_t ts_hi) {
  typedef Mfma<T> MT;
  typedef typename MT::S S;
  __shared__ S Pr[TS][NB + 1], Ps[TS][NB + 1];
  const int j = blockIdx.y;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (k0 >= n) return;
  const int64_t kj = min<int64_t>(kk, n - k0);   // panel columns of this matrix
  const int64_t t0 = k0 + kj;
  const int64_t W = min<int64_t>(B, n - t0);
  if (W <= 0) return;
  const int64_t nt = (W + TS - 1) / TS;
  const int64_t tile = blockIdx.x;
  int64_t tr, ts;
  if (col_only) {
    if (tile >= nt) return;
    tr = tile;
    ts = 0;
  } else {
    // tile columns ts_lo <= ts < ts_hi, each with its rows ts <= tr < nt, column by column
    const int64_t te = min(ts_hi, nt);
    int64_t rem = tile;
    for (ts = ts_lo; ts < te && rem >= nt - ts; ++ts) rem -= nt - ts;
    if (ts >= te) return;
    tr = ts + rem;
  }
  T* base = v + a.off[j];
  const int64_t r0 = t0 + tr * TS, s0 = t0 + ts * TS, wend = t0 + W;
  // thread t loads column t % 64 of rows t / 64 + 4 u (u < 16) of both blocks; loads are
  // unconditional (a masked entry reads a neighbouring band entry: the row index is clamped
  // below n and the allocation is padded past its end) and the mask applies afterwards
  constexpr int L = TS * NB / ST;
  constexpr int RS = ST / NB;                    // rows staged per pass
  const int cl = threadIdx.x % NB, i0 = threadIdx.x / NB;
  const int64_t rs = ld - 1;                     // entry (r, c) at r * rs + B + c
  const int64_t rlast = n - 1;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int rb = 16 * (w & 3), sb = 32 * (w >> 2);
  typename MT::V acc[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) acc[q] = typename MT::V{0, 0, 0, 0};
  for (int64_t kc = 0; kc < kj; kc += NB) {
    const int64_t col = k0 + kc + cl;
    const bool okc = kc + cl < kj;
    S vr[L], vs[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int64_t r = r0 + i0 + RS * u, ss = s0 + i0 + RS * u;
      vr[u] = (S)base[min(r, rlast) * rs + B + col];
      vs[u] = (S)base[min(ss, rlast) * rs + B + col];
    }
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int64_t r = r0 + i0 + RS * u, ss = s0 + i0 + RS * u;
      const bool okr = okc && r < wend && col >= r - B;
      const bool oks = okc && ss < wend && col >= ss - B;
      Pr[i0 + RS * u][cl] = okr ? vr[u] : (S)0;
      Ps[i0 + RS * u][cl] = oks ? vs[u] : (S)0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < NB; k += 4) {
      const S a0 = Pr[rb + li][k + lk];
      const S b0 = Ps[sb + li][k + lk], b1 = Ps[sb + 16 + li][k + lk];
      acc[0] = MT::mma(a0, b0, acc[0]);
      acc[1] = MT::mma(a0, b1, acc[1]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t r = r0 + rb + MT::row(q, lk);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int64_t s = s0 + sb + 16 * t + li;
      if (r < wend && s <= r && (!col_only || s < t0 + TS)) {
        T* e = base + r * ld + (s - r + B);
        *e = (T)((S)*e - acc[t][q]);
      }
    }
  }
}

// Number of tiles k_syrk enumerates for tile columns [lo, hi) of an nt x nt lower triangle.
static unsigned syrk_tiles(int64_t nt, int64_t lo, int64_t hi) {
  int64_t c = 0;
  for (int64_t ts = lo; ts < std::min(hi, nt); ++ts) c += nt - ts;
  return (unsigned)c;
}

template <class T>
void band_factor_t(BandSet& bs, T* v, T* dinv, hipStream_t st, FactorJob& job) {
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p};
  job.inv.alloc((size_t)bs.n_mat * NB * NB);
  double* inv = job.inv.p;
  int* err = job.err.p;
  // right-looking blocked Cholesky in groups of GP panels of NB columns: inside a group
  // each panel is first brought up to date by the group's earlier panels (its own tile
  // column only), then factored (diagonal block, panel below it); the rest of the band is
  // updated once per group, by all GP panels together.  That update is split with
  // look-ahead: the next group's GP tile columns on st, which then goes on to factor that
  // group's panels, and all further tile columns on a second stream at the same time.
  // The next group's own update of the columns after it waits for that second part (the
  // two touch the same tiles); everything else they do touches disjoint tiles.
  constexpr int GP = 4;
  const int64_t nt = (bs.max_B + TS - 1) / TS;
  const unsigned tiles_next = syrk_tiles(nt, 0, GP), tiles_rest = syrk_tiles(nt, GP, nt);
  const unsigned trsm_blocks = (unsigned)((bs.max_B + TS - 1) / TS);
  GX_HIP(hipStreamCreateWithFlags(&job.la, hipStreamNonBlocking));
  GX_HIP(hipEventCreateWithFlags(&job.panels, hipEventDisableTiming));
  GX_HIP(hipEventCreateWithFlags(&job.rest, hipEventDisableTiming));
  bool rest_pending = false;
  for (int64_t k0 = 0; k0 < bs.max_n; k0 += GP * NB) {
    for (int p = 0; p < GP && k0 + p * NB < bs.max_n; ++p) {
      const int64_t c0 = k0 + p * NB;
      if (p > 0 && bs.max_B > 0)
        hipLaunchKernelGGL(k_syrk<T>, dim3((unsigned)nt, bs.n_mat), dim3(ST), 0, st, a, v, k0,
                           (int64_t)p * NB, 1, (int64_t)0, (int64_t)0);
      hipLaunchKernelGGL(k_potrf<T>, dim3(bs.n_mat), dim3(256), 0, st, a, v, c0, inv, dinv,
                         bs.d_boff.p, err);
      if (bs.max_B > 0)
        hipLaunchKernelGGL(k_trsm<T>, dim3(trsm_blocks, bs.n_mat), dim3(256), 0, st, a, v, c0,
                           inv);
    }
    if (bs.max_B > 0) {
      GX_HIP(hipEventRecord(job.panels, st));
      if (tiles_rest) {
        GX_HIP(hipStreamWaitEvent(job.la, job.panels, 0));
        hipLaunchKernelGGL(k_syrk<T>, dim3(tiles_rest, bs.n_mat), dim3(ST), 0, job.la, a, v, k0,
                           (int64_t)GP * NB, 0, (int64_t)GP, nt);
      }
      if (rest_pending) GX_HIP(hipStreamWaitEvent(st, job.rest, 0));
      hipLaunchKernelGGL(k_syrk<T>, dim3(tiles_next, bs.n_mat), dim3(ST), 0, st, a, v, k0,
                         (int64_t)GP * NB, 0, (int64_t)0, (int64_t)GP);
      if (tiles_rest) {
        GX_HIP(hipEventRecord(job.rest, job.la));
        rest_pending = true;
      }
    }
  }
  if (rest_pending) GX_HIP(hipStreamWaitEvent(st, job.rest, 0));
  GX_HIP(hipGetLastError());
}

FactorJob::~FactorJob() {
  if (st) (void)hipStreamSynchronize(st);         // nothing of the job may still run when
  if (la) (void)hipStreamSynchronize(la);         // its buffers are released
  if (panels) (void)hipEventDestroy(panels);
  if (rest) (void)hipEventDestroy(rest);
  if (la) (void)hipStreamDestroy(la);
}

void band_factor_start(BandSet& bs, hipStream_t st, FactorJob& job, const char* what) {
  GX_REQUIRE(!job.st, "factorisation job already started");
  job.st = st;
  job.what = what;
  job.err.alloc(1);
  zero(job.err, st);
  if (bs.fp32)
    band_factor_t<float>(bs, bs.v32.p, bs.dinv32.p, st, job);
  else
    band_factor_t<double>(bs, bs.v64.p, bs.dinv64.p, st, job);
}

void band_factor_finish(FactorJob& job) {
  GX_REQUIRE(job.st, "factorisation job not started");
  int h = 0;
  to_host(&h, job.err.p, 1, job.st);               // waits for all of the job
  if (h)
    throw Error(GX_ENOTSPD,
                "non-positive pivot in the banded Cholesky factorisation of " + job.what);
}

void band_factor(BandSet& bs, hipStream_t st, const char* what) {
  FactorJob job;
  band_factor_start(bs, st, job, what);
  band_factor_finish(job);
}

// ---------------------------------------------------------------------------------------
// Solves: forward L y = b, then backward L^T x = y, in place on FP64 right-hand sides.
// A matrix is swept in blocks of 64 rows.  The coupling between consecutive blocks runs
// through the explicit inverse of each 64x64 diagonal block (kept by the factorisation),
// so the serial part of a block is one small product, not a 64-step substitution.
//
// G work-groups share a matrix: block k belongs to work-group k mod G in the forward sweep
// and to (nblk - 1 - k) mod G in the backward sweep.  A work-group first adds the
// contributions of the blocks that are complete by construction (its own previous block
// and everything before it), then takes the at most G - 1 blocks still in flight from the
// other work-groups (bounded polls of their solutions, below), applies the inverse
// diagonal block and hands its block on.  A timed-out poll raises the launch's error word
// and proceeds, so every wave always reaches the end of the kernel.
constexpr int SW = SOLVE_THREADS / 64;           // waves per work-group (8)
constexpr int RPW = SB / SW;                      // forward rows per wave (8)
constexpr int GMAX = 4;                           // work-groups per matrix, 1-RHS solve
constexpr int DL = SB * SB / SOLVE_THREADS;       // inverse-block entries per thread (8)
static_assert(DL == RPW, "the inverse-block products reuse the 8-row lane reduction");
constexpr int64_t SPIN_LIMIT = (int64_t)1 << 22;
constexpr int64_t BAND_PAD = 1024;               // trailing entries of a band allocation

// Band entry (r, c) loaded from a clamped, always valid address; the caller masks entries
// outside the band.  The loads are unconditional so that a wave issues all of them before
// it waits for any.
template <class T>
__device__ inline T band_raw(const T* base, int64_t n, int64_t B, int64_t ld, int64_t r,
                             int64_t c) {
  const int64_t rc = min(r, n - 1);
  const int64_t o = min(max(c - rc + B, (int64_t)0), B);
  return base[rc * ld + o];
}

// s[r] summed over the 64 lanes; lane l receives the total of row l >> 3
__device__ inline double reduce_rows8(const double (&s)[RPW], int lane) {
  double t4[4], t2[2];
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double send = b5 ? s[r] : s[r + 4];
    t4[r] = (b5 ? s[r + 4] : s[r]) + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const double send = b4 ? t4[r] : t4[r + 2];
    t2[r] = (b4 ? t4[r + 2] : t4[r]) + __shfl_xor(send, 16);
  }
  double t = (b3 ? t2[1] : t2[0]) + __shfl_xor(b3 ? t2[0] : t2[1], 8);
  t += __shfl_xor(t, 4);
  t += __shfl_xor(t, 2);
  t += __shfl_xor(t, 1);
  return t;
}

// ---- one right-hand side per matrix
// Loads are unconditional: rows past the end of the matrix are clamped to its last row, a
// lane whose column lies outside the band reads a neighbouring entry (the band storage
// carries BAND_PAD zero entries after the last row), and masks are applied by multiplying
// with 0 or 1, so that a wave issues all loads of a step before it waits for any.
//
// Hand-over between the work-groups of a matrix goes through the data itself, not flags:
// the forward sweep writes block k's solution into the scratch vector y and the backward
// sweep its final solution into the scratch vector z, both filled with the marker YMARK
// before the launch; a reader of a block that may still be in flight polls its entries
// until none is YMARK, and the values it polled are the ones it uses.  z is copied into x
// after the launch.  Every access to y and z is an agent-scope relaxed atomic (8 bytes,
// single-copy atomic, past the non-coherent caches), so no fence is needed anywhere: a
// hand-over costs the reader one memory round trip and the writer none.  A marker is a NaN
// payload that arithmetic never produces (a NaN result carries the default payload), so a
// diverged solve still propagates NaN.
// COARSE only names the instance used for the coarse matrix apart in profiles.
constexpr uint64_t YMARK = 0x7FF4D1E5E7C0DE00ull;

__device__ inline bool is_mark(double v) { return __double_as_longlong(v) == (long long)YMARK; }

__device__ inline double poll_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void hand_over(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin-limit bookkeeping of a polling loop: true when the wait must give up (time-out, or
// another wait of the launch already timed out).
__device__ inline bool poll_give_up(int64_t& spins, int* err) {
  if ((++spins & 255) == 0 &&
      (spins > SPIN_LIMIT || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
    atomicOr(err, 2);
    return true;
  }
  __builtin_amdgcn_s_sleep(1);
  return false;
}

// Work-group g of the G that solve one matrix of n rows, half-bandwidth B and row stride
// ld: factor from base, inverse diagonal blocks from dv, right-hand side x, scratch y, z.
template <class T>
__device__ __forceinline__ void band_solve_1_mat(int64_t n, int64_t B, int64_t ld,
                                                 const T* base, const T* dv, const double* x,
                                                 double* y, double* z, int g, int G, int* err) {
  __shared__ double acc[SB];
  __shared__ double part[SW][SB];
  __shared__ double xs[GMAX - 1][SB];               // polled solutions of blocks in flight
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nblk = (n + SB - 1) / SB;
  constexpr int U = 8;                             // 64-column steps in flight per wave
  constexpr int UB = 32;                           // band rows in flight per wave (backward)
  // ---- forward: wave w owns rows 8w..8w+7 of the block, lanes run along the columns
  for (int64_t k = g; k < nblk; k += G) {
    const int64_t i0 = k * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t kdone = max<int64_t>(k - G + 1, 0);        // column blocks < kdone complete
    const int64_t done_end = kdone * SB;
    const int64_t ifirst = i0 + RPW * wave;
    // the right-hand side of the row this lane reduces
    const int ii = RPW * wave + (lane >> 3);
    const bool own = (lane & 7) == 0 && ii < nb;
    const double bval = own ? x[i0 + ii] : 0.0;
    const T* rp[RPW];                              // rp[r][c] = entry (row, c)
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int64_t rc = min<int64_t>(ifirst + r, n - 1);
      rp[r] = base + rc * ld - rc + B;
    }
    double s[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) s[r] = 0.0;
    for (int64_t c0 = max<int64_t>(ifirst - B, 0) + lane; c0 < done_end + lane; c0 += 64 * U) {
      T l[U][RPW];
      double xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        xv[u] = poll_load(y + min<int64_t>(c0 + 64 * u, done_end - 1));
#pragma unroll
        for (int r = 0; r < RPW; ++r) l[u][r] = rp[r][c0 + 64 * u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t cc = c0 + 64 * u;
        const double xu = cc < done_end ? xv[u] : 0.0;
#pragma unroll
        for (int r = 0; r < RPW; ++r)
          s[r] += (double)l[u][r] * (cc >= ifirst + r - B ? xu : 0.0);
      }
    }
    // blocks in flight, kdone .. k - 1 (at most GMAX - 1): their factor entries and this
    // block's inverse diagonal block are loaded first; then wave 0 polls their solutions
    // (one round trip when they are done) and passes them on through LDS
    const int nfl = (int)(k - kdone);
    T pf[GMAX - 1][RPW], dd[DL];
#pragma unroll
    for (int o = 0; o < GMAX - 1; ++o) {
      const int64_t cc = min<int64_t>(kdone + o, max<int64_t>(k - 1, 0)) * SB + lane;
#pragma unroll
      for (int r = 0; r < RPW; ++r) pf[o][r] = rp[r][cc];
    }
#pragma unroll
    for (int u = 0; u < DL; ++u) dd[u] = dv[k * SB * SB + threadIdx.x + SOLVE_THREADS * u];
    if (nfl > 0) {
      if (wave == 0) {
        double xo[GMAX - 1];
        int64_t spins = 0;
        for (;;) {
          bool ok = true;
#pragma unroll
          for (int o = 0; o < GMAX - 1; ++o) {
            xo[o] = poll_load(y + min<int64_t>(kdone + o, k - 1) * SB + lane);
            ok = ok && !is_mark(xo[o]);
          }
          if (__all(ok) || poll_give_up(spins, err)) break;
        }
#pragma unroll
        for (int o = 0; o < GMAX - 1; ++o) xs[o][lane] = xo[o];
      }
      __syncthreads();
      double xo[GMAX - 1];
#pragma unroll
      for (int o = 0; o < GMAX - 1; ++o) xo[o] = xs[o][lane];
#pragma unroll
      for (int o = 0; o < GMAX - 1; ++o) {
        if (o >= nfl) break;
        const int64_t cc = (kdone + o) * SB + lane;
#pragma unroll
        for (int r = 0; r < RPW; ++r)
          s[r] += (double)pf[o][r] * (cc >= ifirst + r - B ? xo[o] : 0.0);
      }
    }
    const double tot = reduce_rows8(s, lane);
    if ((lane & 7) == 0) acc[ii] = own ? bval - tot : 0.0;
    __syncthreads();
    // y = Di acc: thread (wave, lane) holds Di[wave + 8 u][lane] (u < 8) from the prefetch,
    // so each wave forms rows wave + 8 u with one lane-wide reduction
    {
      const double av = acc[lane];
      double pr[RPW];
#pragma unroll
      for (int u = 0; u < DL; ++u) pr[u] = (double)dd[u] * av;
      const double yr = reduce_rows8(pr, lane);
      const int row = wave + SW * (lane >> 3);
      if ((lane & 7) == 0 && row < nb) hand_over(y + i0 + row, yr);
    }
    __syncthreads();
  }
  // ---- backward: lanes own the block's 64 columns, waves split the band rows below it;
  // entry (r, c) = cb[r * rs + c]
  const T* cb = base + B;
  const int64_t rs = ld - 1;
  for (int64_t t = g; t < nblk; t += G) {
    const int64_t kb = nblk - 1 - t;
    const int64_t i0 = kb * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t rend = min<int64_t>(n, i0 + nb + B);
    const int64_t kdone = kb + G;                  // row blocks >= kdone complete
    const int64_t done_beg = min<int64_t>(rend, kdone * SB);
    const int64_t cidx = i0 + lane;
    double sacc = 0.0;
    for (int64_t r0 = done_beg + wave; r0 < rend; r0 += SW * UB) {
      // lane u < UB loads the solution of row r0 + 8 u, handed to all lanes by a lane read
      T l[UB];
      const double xz = poll_load(z + min<int64_t>(r0 + SW * (lane % UB), rend - 1));
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int64_t rr = min<int64_t>(r0 + SW * u, rend - 1);
        l[u] = cb[rr * rs + cidx];
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int64_t rr = r0 + SW * u;
        const double xu = __shfl(xz, u);
        sacc += (double)l[u] * ((rr < rend && rr - B <= cidx) ? xu : 0.0);
      }
    }
    // row blocks in flight, kb + 1 .. kin (at most GMAX - 1): factor entries and the
    // inverse diagonal block first, then the polls of their final solutions (rows inside
    // the band only) together with this block's forward solution
    const int64_t kin = min<int64_t>(kdone - 1, (rend - 1) / SB);   // last row block in flight
    const int nfl = (int)max<int64_t>(kin - kb, 0);
    T pf[GMAX - 1][RPW], dd[DL];
#pragma unroll
    for (int o = 0; o < GMAX - 1; ++o)
#pragma unroll
      for (int r = 0; r < RPW; ++r)
        pf[o][r] = cb[min<int64_t>((kb + 1 + o) * SB + wave + SW * r, n - 1) * rs + cidx];
#pragma unroll
    for (int u = 0; u < DL; ++u) dd[u] = dv[kb * SB * SB + threadIdx.x + SOLVE_THREADS * u];
    // wave 0 polls this block's forward solution and the final solutions of the rows in
    // flight (lane l: row l of each block), and passes them on through LDS
    double yown = 0.0;
    if (wave == 0) {
      double xo[GMAX - 1];
      int64_t spins = 0;
      for (;;) {
        bool ok = true;
        if (lane < nb) {
          yown = poll_load(y + cidx);
          ok = !is_mark(yown);
        }
#pragma unroll
        for (int o = 0; o < GMAX - 1; ++o) {
          const int64_t rr = (kb + 1 + o) * SB + lane;
          const bool need = o < nfl && rr < rend;
          xo[o] = poll_load(z + min<int64_t>(rr, rend - 1));
          ok = ok && (!need || !is_mark(xo[o]));
        }
        if (__all(ok) || poll_give_up(spins, err)) break;
      }
#pragma unroll
      for (int o = 0; o < GMAX - 1; ++o) xs[o][lane] = xo[o];
    }
    __syncthreads();
    double xr[GMAX - 1][RPW];
#pragma unroll
    for (int o = 0; o < GMAX - 1; ++o)
#pragma unroll
      for (int r = 0; r < RPW; ++r) xr[o][r] = xs[o][wave + SW * r];
#pragma unroll
    for (int o = 0; o < GMAX - 1; ++o) {
      if (o >= nfl) break;
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int64_t rr = (kb + 1 + o) * SB + wave + SW * r;
        sacc += (double)pf[o][r] * ((rr < rend && rr - B <= cidx) ? xr[o][r] : 0.0);
      }
    }
    part[wave][lane] = sacc;
    if (wave == 0) acc[lane] = lane < nb ? yown : 0.0;
    __syncthreads();
    // z = Di^T (yown - sums): thread (wave, lane) holds Di[wave + 8 u][lane]; each wave
    // forms its rows' right-hand sides (broadcast reads), then its share of every column
    {
      double pc = 0.0;
#pragma unroll
      for (int u = 0; u < DL; ++u) {
        const int r = wave + SW * u;
        double t = acc[r];
#pragma unroll
        for (int w = 0; w < SW; ++w) t -= part[w][r];
        pc += (double)dd[u] * (r < nb ? t : 0.0);
      }
      __syncthreads();
      part[wave][lane] = pc;
    }
    __syncthreads();
    if (wave == 0) {
      double zs = 0.0;
#pragma unroll
      for (int w = 0; w < SW; ++w) zs += part[w][lane];
      if (lane < nb) hand_over(z + cidx, zs);
    }
    __syncthreads();
  }
}

// Matrices j of one band set: work-group (g, j) at blockIdx.x = g * n_pad + j.
template <class T, bool COARSE>
__global__ void __launch_bounds__(SOLVE_THREADS) k_band_solve_1(
    BandArgs a, const T* v, const T* dinv, const int64_t* boff, const int64_t* xoff,
    const double* xall, double* yall, double* zall, const int64_t* yoff, int G, int n_pad,
    int n_mat, int* err) {
  const int g = blockIdx.x / n_pad, j = blockIdx.x % n_pad;
  if (j >= n_mat || g >= G) return;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (n == 0) return;
  band_solve_1_mat<T>(n, B, ld, v + a.off[j], dinv + boff[j], xall + xoff[j], yall + yoff[j],
                      zall + yoff[j], g, G, err);
}

// The matrices of several band sets in one launch (all of one precision): work-group i
// takes group work[2 i + 1] of matrix work[2 i] (none if negative); matrix j's rows,
// bandwidth, group count, factor, inverse diagonal blocks, right-hand side and scratch
// come from tab[j].
template <class T>
__global__ void __launch_bounds__(SOLVE_THREADS) k_band_solve_1_multi(const BandPtrs* tab,
                                                                       const int32_t* work,
                                                                       int* err) {
  const int j = work[2 * blockIdx.x], g = work[2 * blockIdx.x + 1];
  if (j < 0) return;
  const BandPtrs t = tab[j];
  if (t.n == 0) return;
  band_solve_1_mat<T>(t.n, t.B, t.B + 1, static_cast<const T*>(t.v),
                      static_cast<const T*>(t.dinv), t.x, t.y, t.z, g, (int)t.G, err);
}

// y and z scratch of every matrix of a multi-set solve back to the marker
__global__ void k_fill_mark_multi(const BandPtrs* tab) {
  const BandPtrs t = tab[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (t.n + SB - 1) / SB * SB) {
    t.y[i] = __longlong_as_double((long long)YMARK);
    t.z[i] = __longlong_as_double((long long)YMARK);
  }
}

// x_j <- z_j for every matrix of a multi-set solve
__global__ void k_copy_out_multi(const BandPtrs* tab) {
  const BandPtrs t = tab[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < t.n) t.x[i] = t.z[i];
}

// ---- M right-hand sides per matrix (M a multiple of 8, at most MC; row-major, row
// stride M)
// The block products - a 64-row block of the band against 64 solution rows, and the
// inverse diagonal block against the block's right-hand side - are 64 x 64 x M and run on
// FP64 matrix cores: v_mfma_f64_16x16x4, lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 r + l / 16][l % 16] in accumulator register r; wave w
// of the 8 owns row tile w mod 4 and column tile w / 4.  Chunks (64 x 64 of the band plus
// the matching solution rows) are staged through two LDS buffers in turn; the loads of the
// next two chunks are in flight in two register sets while the current one is multiplied
// (the chunk loop is unrolled by two so that each set and buffer has a name of its own).
// Hand-over between work-groups
// goes through marker-filled scratch solutions as in the single-right-hand-side solve
// (forward into y, backward into z, z copied into x afterwards): solution entries are
// loaded with agent-scope relaxed atomics, and a chunk is staged only once none of the
// entries it needs is a marker (a chunk still in flight is polled again until then).
constexpr int MC = 32;                            // right-hand sides per launch, at most
constexpr int MT = 512;                           // threads per work-group
constexpr int AL = SB * SB / MT;                  // band-chunk entries per thread (8)

template <class T, int M>
__global__ void __launch_bounds__(MT) k_band_solve_m(
    BandArgs a, const T* v, const T* dinv, const int64_t* boff, const int64_t* xoff,
    const double* xall, double* yall, double* zall, const int64_t* yoff, int G, int n_pad,
    int n_mat, const int32_t* active, int* err) {
  typedef Mfma<T> MF;
  typedef typename MF::S S;
  constexpr int NCT = (M + 15) / 16;              // column tiles (1 or 2)
  constexpr int MP = 16 * NCT;                    // LDS row stride (zero columns past M)
  constexpr int YL = SB * M / MT;                 // solution-chunk entries per thread
  __shared__ S Ab[2][SB][SB + 1];                 // band chunks (double buffer); buffer 0
  __shared__ S Yc[2][SB * MP];                    // holds the inverse block in finish
  const int g = blockIdx.x / n_pad, j = blockIdx.x % n_pad;
  if (j >= n_mat || g >= G) return;
  if (active && !active[j]) return;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (n == 0) return;
  const T* cb = v + a.off[j] + B;                 // entry (r, c) = cb[r * rs + c]
  const int64_t rs = ld - 1;
  const T* dv = dinv + boff[j];
  const double* x = xall + xoff[j];
  double* y = yall + yoff[j] * M;
  double* z = zall + yoff[j] * M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rt = wave & 3, ct = wave >> 2;        // this wave's row and column tile
  const bool tile = ct < NCT;                      // waves past the column tiles only stage
  const int li = lane & 15, lk = lane >> 4;
  const int64_t nblk = (n + SB - 1) / SB;
  if constexpr (MP > M)
    for (int idx = threadIdx.x; idx < 2 * SB * (MP - M); idx += MT) {
      const int e = idx % (SB * (MP - M));
      Yc[idx / (SB * (MP - M))][(e / (MP - M)) * MP + M + e % (MP - M)] = (S)0;
    }
  // forward chunk kk of block i0: band rows i0.., columns 64 kk..; backward chunk kk:
  // band rows 64 kk.., columns i0..; both with solution rows 64 kk..  Thread t stages band
  // rows t / 64 + 8 u at column t % 64.
  auto fetch = [&](bool bwd, int64_t i0, int64_t kk, T (&fa)[AL], double (&fy)[YL]) {
    const int64_t r0 = (bwd ? kk * SB : i0) + wave;
    const int64_t c = (bwd ? i0 : kk * SB) + lane;
#pragma unroll
    for (int u = 0; u < AL; ++u) fa[u] = cb[min<int64_t>(r0 + 8 * u, n - 1) * rs + c];
    const int64_t yend = min<int64_t>((int64_t)SB * M, (n - kk * SB) * M);   // rows < n
    const double* xs = (bwd ? z : y) + kk * SB * M;
#pragma unroll
    for (int u = 0; u < YL; ++u) fy[u] = poll_load(xs + min<int64_t>(threadIdx.x + MT * u, yend - 1));
  };
  auto stage = [&](int buf, bool bwd, int64_t i0, int nb, int64_t kk, const T (&fa)[AL],
                   double (&fy)[YL]) {
    {                                              // until every needed entry is handed over
      const int64_t yend = min<int64_t>((int64_t)SB * M, (n - kk * SB) * M);
      const double* xs = (bwd ? z : y) + kk * SB * M;
      // the first test on the values already loaded is straight-line code, so the wait
      // before it covers only this chunk's loads, not the prefetch of the next one; the
      // polling loop is the slow path of a chunk still in flight
      bool ok = true;
#pragma unroll
      for (int u = 0; u < YL; ++u) ok = ok && (threadIdx.x + MT * u >= yend || !is_mark(fy[u]));
      if (!__all(ok)) {
        int64_t spins = 0;
        for (;;) {
          if (poll_give_up(spins, err)) break;
#pragma unroll
          for (int u = 0; u < YL; ++u)
            fy[u] = poll_load(xs + min<int64_t>(threadIdx.x + MT * u, yend - 1));
          bool again = false;
#pragma unroll
          for (int u = 0; u < YL; ++u)
            again = again || (threadIdx.x + MT * u < yend && is_mark(fy[u]));
          if (!__any(again)) break;
        }
      }
    }
    const int64_t r0 = (bwd ? kk * SB : i0) + wave;
    const int64_t c = (bwd ? i0 : kk * SB) + lane;
#pragma unroll
    for (int u = 0; u < AL; ++u) {
      const int64_t r = r0 + 8 * u;
      const bool in = r < n && c <= r && c >= r - B && (!bwd || lane < nb);
      Ab[buf][wave + 8 * u][lane] = in ? (S)fa[u] : (S)0;
    }
    const int64_t yend = min<int64_t>((int64_t)SB * M, (n - kk * SB) * M);   // rows < n
#pragma unroll
    for (int u = 0; u < YL; ++u) {
      const int idx = threadIdx.x + MT * u;
      Yc[buf][(idx / M) * MP + idx % M] = idx < yend ? (S)fy[u] : (S)0;
    }
  };
  // acc += A Yc over the 64-deep chunk for this wave's tile; A = Ab or Ab^T.  Even and odd
  // 4-deep steps go to two accumulators, so consecutive matrix instructions do not wait
  // for each other's result.
  auto mma = [&](int buf, bool trans, typename MF::V& acc) {
    if (!tile) return;
    typename MF::V acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < SB / 4; ks += 2) {
      const int kq0 = 4 * ks + lk, kq1 = kq0 + 4;
      const S a0 = trans ? Ab[buf][kq0][16 * rt + li] : Ab[buf][16 * rt + li][kq0];
      const S a1 = trans ? Ab[buf][kq1][16 * rt + li] : Ab[buf][16 * rt + li][kq1];
      const S b0 = Yc[buf][kq0 * MP + 16 * ct + li];
      const S b1 = Yc[buf][kq1 * MP + 16 * ct + li];
      acc = MF::mma(a0, b0, acc);
      acc1 = MF::mma(a1, b1, acc1);
    }
    acc += acc1;
  };
  // the chunks kk = first, first + step, .., last (step +1 or -1): chunk q is multiplied
  // from LDS buffer q % 2 while its loads were issued two chunks earlier; each wave stages
  // chunk q + 1 into the other buffer right after its product of chunk q, so one barrier
  // per chunk separates the staging of a buffer from its readers (the product two chunks
  // back, and the next product)
  auto sweep = [&](bool bwd, int64_t i0, int nb, int64_t first, int64_t count, int step,
                   typename MF::V& acc) {
    if (count <= 0) return;
    T fa0[AL], fa1[AL];
    double fy0[YL], fy1[YL];
    // chunk q, clamped to the last one: every prefetch is issued unconditionally (a chunk
    // past the end repeats the last, never used), which keeps the loads in flight the same
    // on every path and lets each wait count only the chunk it needs
    const int64_t qmax = count - 1;
    auto kk_of = [&](int64_t q) { return first + step * min(q, qmax); };
    fetch(bwd, i0, kk_of(0), fa0, fy0);
    fetch(bwd, i0, kk_of(1), fa1, fy1);
    __syncthreads();                               // finish of the last block read buffer 0
    stage(0, bwd, i0, nb, kk_of(0), fa0, fy0);
    for (int64_t q = 0; q < count; q += 2) {
      __syncthreads();
      fetch(bwd, i0, kk_of(q + 2), fa0, fy0);
      mma(0, bwd, acc);
      if (q + 1 >= count) break;
      stage(1, bwd, i0, nb, kk_of(q + 1), fa1, fy1);
      __syncthreads();
      fetch(bwd, i0, kk_of(q + 3), fa1, fy1);
      mma(1, bwd, acc);
      stage(0, bwd, i0, nb, kk_of(q + 2), fa0, fy0);
    }
  };
  // Yc <- rhs - accumulated sums (rows >= nb zero), Ab <- inverse block; the product with
  // it is the block's solution, handed over.  The right-hand side is x forward and the
  // block's forward solution (polled) backward.
  // (dd: the block's inverse diagonal block, loaded before the sweep so that its latency
  // stays off the chain of hand-overs)
  auto finish = [&](bool bwd, int64_t i0, int nb, const T (&dd)[AL],
                    const typename MF::V& acc) {
    double bb[4];
    const int cc = min(16 * ct + li, M - 1);
    if (!bwd) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = min<int64_t>(i0 + 16 * rt + MF::row(r, lk), n - 1);
        bb[r] = x[row * M + cc];
      }
    } else {
      int64_t spins = 0;
      for (;;) {
        bool ok = true;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ii = 16 * rt + MF::row(r, lk);
          bb[r] = poll_load(y + (i0 + min(ii, nb - 1)) * M + cc);
          ok = ok && (!tile || ii >= nb || !is_mark(bb[r]));
        }
        if (__all(ok) || poll_give_up(spins, err)) break;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < AL; ++u) {
      const int idx = threadIdx.x + MT * u;
      Ab[0][idx >> 6][idx & 63] = (S)dd[u];
    }
    if (tile)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = 16 * rt + MF::row(r, lk), col = 16 * ct + li;
        if (col < M) Yc[0][ii * MP + col] = ii < nb ? (S)(bb[r] - (double)acc[r]) : (S)0;
      }
    __syncthreads();
    typename MF::V yv = {0, 0, 0, 0};
    mma(0, bwd, yv);
    double* dst = bwd ? z : y;
    if (tile)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = 16 * rt + MF::row(r, lk), col = 16 * ct + li;
        if (ii < nb && col < M) hand_over(dst + (i0 + ii) * M + col, (double)yv[r]);
      }
    __syncthreads();
  };
  // ---- forward: chunks in increasing order; those from kdone on are still in flight
  for (int64_t k = g; k < nblk; k += G) {
    const int64_t i0 = k * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t kfirst = max<int64_t>(i0 - B, 0) / SB;
    T dd[AL];
#pragma unroll
    for (int u = 0; u < AL; ++u) dd[u] = dv[k * SB * SB + threadIdx.x + MT * u];
    typename MF::V acc = {0, 0, 0, 0};
    sweep(false, i0, nb, kfirst, k - kfirst, 1, acc);
    finish(false, i0, nb, dd, acc);
  }
  // ---- backward: chunks from the far end of the band inwards
  for (int64_t t = g; t < nblk; t += G) {
    const int64_t kb = nblk - 1 - t;
    const int64_t i0 = kb * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t klast = (min<int64_t>(n, i0 + nb + B) - 1) / SB;   // last row block
    T dd[AL];
#pragma unroll
    for (int u = 0; u < AL; ++u) dd[u] = dv[kb * SB * SB + threadIdx.x + MT * u];
    typename MF::V acc = {0, 0, 0, 0};
    sweep(true, i0, nb, klast, klast - kb, -1, acc);
    finish(true, i0, nb, dd, acc);
  }
}

// Work-groups per matrix: as many as keep every work-group of the launch resident at once
// (the waits rely on it); at most GMAX for one right-hand side, 8 for several.  The solves
// of one context are stream-ordered, so a launch may count on the whole machine (other
// kernels can only delay the dispatch of its groups, not block them).  When several
// contexts solve concurrently (share > 1) each gets an equal part of three quarters of it,
// so that all their launches fit together.
static int solve_groups(BandSet& bs, const void* kernel, int which) {
  if (bs.solve_groups[which] > 0) return bs.solve_groups[which];
  int dev = 0, cus = 0, per_cu = 0;
  GX_HIP(hipGetDevice(&dev));
  GX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  GX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel,
                                                      which == 0 ? SOLVE_THREADS : MT, 0));
  const int64_t full = (int64_t)cus * std::max(per_cu, 0);
  const int64_t capacity = bs.share > 1 ? full * 3 / 4 / bs.share : full;
  const int cap = which == 0 ? GMAX : 8;
  int G = 1;
  const int top = bs.force_groups[which] > 0 ? std::min(bs.force_groups[which], cap) : cap;
  for (int c = top; c >= 2; --c)
    if ((int64_t)bs.n_mat * c <= capacity && bs.max_n >= (int64_t)2 * SB * c) {
      G = c;
      break;
    }
  bs.solve_groups[which] = G;
  return G;
}

// The launch's error word (raised by a poll that timed out), zero until a check clears it
static int* solve_err(BandSet& bs, hipStream_t st, int& n_pad) {
  n_pad = (bs.n_mat + 7) / 8 * 8;                  // all groups of a matrix on one XCD
  if (!bs.err.n) {
    bs.err.alloc(1);
    zero(bs.err, st);
  }
  return bs.err.p;
}

__global__ void k_fill_mark(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = __longlong_as_double((long long)YMARK);
}

// The forward and backward solution scratch of the single-right-hand-side solve (y, then
// z, 64-aligned segments per matrix), reset to the marker by a fill kernel on the stream
// (so the launch can be captured in a graph).
static void alloc_solve1_scratch(BandSet& bs, hipStream_t st) {
  if (bs.d_yoff.n) return;
  std::vector<int64_t> yo(bs.n_mat + 1, 0);
  for (int j = 0; j < bs.n_mat; ++j) yo[j + 1] = yo[j] + (bs.n[j] + SB - 1) / SB * SB;
  bs.ybuf.alloc(2 * std::max<int64_t>(yo[bs.n_mat], 1));
  bs.d_yoff.alloc(bs.n_mat + 1);
  to_dev(bs.d_yoff.p, yo.data(), bs.n_mat + 1, st);
  GX_HIP(hipStreamSynchronize(st));                // yo is a local host vector
}

static double* solve1_scratch(BandSet& bs, hipStream_t st) {
  alloc_solve1_scratch(bs, st);
  hipLaunchKernelGGL(k_fill_mark, dim3(nblocks((int64_t)bs.ybuf.n, 256)), dim3(256), 0, st,
                     bs.ybuf.p, (int64_t)bs.ybuf.n);
  return bs.ybuf.p;
}

// x_j <- z_j for every matrix (the solutions out of the scratch)
__global__ void k_copy_out(const int64_t* nrows, const int64_t* xoff, const int64_t* yoff,
                           const double* z, double* x) {
  const int j = blockIdx.y;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nrows[j]) x[xoff[j] + i] = z[yoff[j] + i];
}

// z_j -> x_j for the active matrices (n_j rows of w columns)
__global__ void k_copy_out_m(const int64_t* nrows, const int64_t* xoff, const int64_t* yoff,
                             int w, const double* z, double* x, const int32_t* active) {
  const int j = blockIdx.y;
  if (active && !active[j]) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nrows[j] * w) x[xoff[j] + i] = z[yoff[j] * w + i];
}

template <int M>
static void launch_m(BandSet& bs, const BandArgs& a, const int64_t* d_xoff, double* x,
                     hipStream_t st, const int32_t* active) {
  const int G = bs.fp32 ? solve_groups(bs, reinterpret_cast<const void*>(&k_band_solve_m<float, M>), 1)
                        : solve_groups(bs, reinterpret_cast<const void*>(&k_band_solve_m<double, M>), 1);
  int n_pad = 0;
  int* err = solve_err(bs, st, n_pad);
  // y and z scratch of M columns: segments at yoff[j] * M rows (64-aligned row offsets)
  if (!bs.d_yoff.n) (void)solve1_scratch(bs, st);
  const int64_t rows = (int64_t)bs.ybuf.n / 2;     // padded rows of all matrices
  if (bs.mbuf.n < (size_t)(2 * rows * MC)) bs.mbuf.alloc(2 * rows * MC);
  hipLaunchKernelGGL(k_fill_mark, dim3(nblocks(2 * rows * M, 256)), dim3(256), 0, st, bs.mbuf.p,
                     2 * rows * M);
  double* y = bs.mbuf.p;
  double* z = bs.mbuf.p + rows * M;
  if (bs.fp32)
    hipLaunchKernelGGL((k_band_solve_m<float, M>), dim3(G * n_pad), dim3(MT), 0, st, a, bs.v32.p,
                       bs.dinv32.p, bs.d_boff.p, d_xoff, x, y, z, bs.d_yoff.p, G, n_pad,
                       bs.n_mat, active, err);
  else
    hipLaunchKernelGGL((k_band_solve_m<double, M>), dim3(G * n_pad), dim3(MT), 0, st, a,
                       bs.v64.p, bs.dinv64.p, bs.d_boff.p, d_xoff, x, y, z, bs.d_yoff.p, G,
                       n_pad, bs.n_mat, active, err);
  hipLaunchKernelGGL(k_copy_out_m, dim3(nblocks(bs.max_n * M, 256), bs.n_mat), dim3(256), 0, st,
                     bs.d_n.p, d_xoff, bs.d_yoff.p, M, z, x, active);
}

// Columns c0 .. c0 + w of a row-major block of ncol columns to or from a contiguous panel
// of w columns (panel of matrix j at poff[j]).
__global__ void k_panel_copy(const int64_t* nrows, const int64_t* xoff, double* x, int ncol,
                             int c0, int w, const int64_t* poff, double* panel,
                             const int32_t* active, int to_panel) {
  const int j = blockIdx.y;
  if (active && !active[j]) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows[j] * w) return;
  const int64_t r = e / w, c = e - r * w;
  double* xe = x + xoff[j] + r * ncol + c0 + c;
  double* pe = panel + poff[j] + e;
  if (to_panel)
    *pe = *xe;
  else
    *xe = *pe;
}

void band_solve(BandSet& bs, const int64_t* d_xoff, double* x, hipStream_t st, int ncol,
                const int32_t* active) {
  GX_REQUIRE(ncol == 1 || (ncol % 8 == 0 && ncol <= 2 * MC),
             "banded solve: right-hand sides must be 1 or a multiple of 8 up to 64");
  if (ncol > MC) {
    // panels of at most MC columns through a scratch block; the factor is read once per panel
    if (!bs.d_poff.n) {
      std::vector<int64_t> po(bs.n_mat + 1, 0);
      for (int j = 0; j < bs.n_mat; ++j) po[j + 1] = po[j] + bs.n[j] * MC;
      bs.panel.alloc(po[bs.n_mat]);
      bs.d_poff.alloc(bs.n_mat + 1);
      to_dev(bs.d_poff.p, po.data(), bs.n_mat + 1, st);
    }
    for (int c0 = 0; c0 < ncol; c0 += MC) {
      const int w = std::min(MC, ncol - c0);
      const dim3 grid(nblocks((int64_t)bs.max_n * w, 256), bs.n_mat);
      hipLaunchKernelGGL(k_panel_copy, grid, dim3(256), 0, st, bs.d_n.p, d_xoff, x, ncol, c0,
                         w, bs.d_poff.p, bs.panel.p, active, 1);
      band_solve(bs, bs.d_poff.p, bs.panel.p, st, w, active);
      hipLaunchKernelGGL(k_panel_copy, grid, dim3(256), 0, st, bs.d_n.p, d_xoff, x, ncol, c0,
                         w, bs.d_poff.p, bs.panel.p, active, 0);
    }
    GX_HIP(hipGetLastError());
    return;
  }
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p};
  int n_pad = 0;
  if (ncol == 1 && !active) {
    const void* kf = bs.fp32 ? reinterpret_cast<const void*>(&k_band_solve_1<float, false>)
                   : bs.coarse ? reinterpret_cast<const void*>(&k_band_solve_1<double, true>)
                               : reinterpret_cast<const void*>(&k_band_solve_1<double, false>);
    const int G = solve_groups(bs, kf, 0);
    int* err = solve_err(bs, st, n_pad);
    double* y = solve1_scratch(bs, st);
    double* z = y + bs.ybuf.n / 2;
    if (bs.fp32)
      hipLaunchKernelGGL((k_band_solve_1<float, false>), dim3(G * n_pad), dim3(SOLVE_THREADS), 0,
                         st, a, bs.v32.p, bs.dinv32.p, bs.d_boff.p, d_xoff, x, y, z,
                         bs.d_yoff.p, G, n_pad, bs.n_mat, err);
    else if (bs.coarse)
      hipLaunchKernelGGL((k_band_solve_1<double, true>), dim3(G * n_pad), dim3(SOLVE_THREADS), 0,
                         st, a, bs.v64.p, bs.dinv64.p, bs.d_boff.p, d_xoff, x, y, z,
                         bs.d_yoff.p, G, n_pad, bs.n_mat, err);
    else
      hipLaunchKernelGGL((k_band_solve_1<double, false>), dim3(G * n_pad), dim3(SOLVE_THREADS), 0,
                         st, a, bs.v64.p, bs.dinv64.p, bs.d_boff.p, d_xoff, x, y, z,
                         bs.d_yoff.p, G, n_pad, bs.n_mat, err);
    hipLaunchKernelGGL(k_copy_out, dim3(nblocks(bs.max_n, 256), bs.n_mat), dim3(256), 0, st,
                       bs.d_n.p, d_xoff, bs.d_yoff.p, z, x);
  } else {
    switch (ncol) {
      case 8: launch_m<8>(bs, a, d_xoff, x, st, active); break;
      case 16: launch_m<16>(bs, a, d_xoff, x, st, active); break;
      case 24: launch_m<24>(bs, a, d_xoff, x, st, active); break;
      default: launch_m<32>(bs, a, d_xoff, x, st, active); break;
    }
  }
  GX_HIP(hipGetLastError());
}

// Algorithmic bytes of one solve: the factor and the inverse diagonal blocks read once per
// sweep, the FP64 right-hand sides read and written once per sweep.
double band_solve_bytes(const BandSet& bs, int ncol, const int32_t* active_host, bool band) {
  const double w = bs.fp32 ? 4.0 : 8.0;
  double b = 0.0;
  for (int j = 0; j < bs.n_mat; ++j) {
    if (active_host && !active_host[j]) continue;
    const double nblk = (double)((bs.n[j] + SB - 1) / SB);
    const double factor = band ? (double)bs.n[j] * (double)(bs.B[j] + 1) + nblk * SB * SB
                               : (double)bs.env[j];
    b += 2.0 * w * factor + 4.0 * 8.0 * (double)bs.n[j] * ncol;
  }
  return b;
}

double band_factor_flops(const BandSet& bs) {
  double f = 0.0;
  for (int j = 0; j < bs.n_mat; ++j) {
    const double n = (double)bs.n[j], B = (double)bs.B[j];
    // columns 0 .. n - 1 - B have w = B; the last B columns have w = B - 1 .. 0
    const double full = std::max(0.0, n - B);
    const double tail = std::min(n, B);                  // w = tail - 1 .. 0
    f += full * (B * B + 2.0 * B + 1.0);
    f += (tail - 1.0) * tail * (2.0 * tail - 1.0) / 6.0 + (tail - 1.0) * tail + tail;
  }
  return f;
}

// The table of a multi-set solve: matrix j of set k solves in place on x[k] + xoff[k][j]
// (xoff[k]: host offsets of set k's right-hand-side segments).  Synchronises st.
void multi_solve_plan(MultiSolve& m, const std::vector<BandSet*>& sets,
                      const std::vector<double*>& x, const std::vector<const int64_t*>& xoff,
                      hipStream_t st) {
  GX_REQUIRE(!sets.empty() && x.size() == sets.size() && xoff.size() == sets.size(),
             "multi-set solve: one right-hand side and offset list per band set");
  GX_HIP(hipStreamSynchronize(st));                // earlier launches may still read the table
  m.sets = sets;
  m.fp32 = sets[0]->fp32;
  m.host.clear();
  m.max_n = 0;
  for (size_t k = 0; k < sets.size(); ++k) {
    BandSet& bs = *sets[k];
    GX_REQUIRE(bs.fp32 == m.fp32 && !bs.coarse && x[k] && xoff[k],
               "multi-set solve: band sets of one precision with right-hand sides");
    alloc_solve1_scratch(bs, st);
    const int64_t half = (int64_t)bs.ybuf.n / 2;
    int64_t yo = 0;
    for (int j = 0; j < bs.n_mat; ++j) {
      BandPtrs t;
      t.v = m.fp32 ? static_cast<const void*>(bs.v32.p + bs.off[j])
                   : static_cast<const void*>(bs.v64.p + bs.off[j]);
      t.dinv = m.fp32 ? static_cast<const void*>(bs.dinv32.p + bs.boff[j])
                      : static_cast<const void*>(bs.dinv64.p + bs.boff[j]);
      t.x = x[k] + xoff[k][j];
      t.y = bs.ybuf.p + yo;
      t.z = bs.ybuf.p + half + yo;
      t.n = bs.n[j];
      t.B = bs.B[j];
      yo += (bs.n[j] + SB - 1) / SB * SB;
      m.max_n = std::max(m.max_n, bs.n[j]);
      m.host.push_back(t);
    }
  }
  m.n_mat = (int)m.host.size();
  GX_REQUIRE(m.n_mat > 0 && m.n_mat <= 65535, "multi-set solve: 1 to 65535 matrices");
  // Work-groups per matrix.  The waits between the groups of a matrix need them all
  // resident, and work-group i runs on XCD i mod NX (each with its share of the resident
  // capacity).  Matrices go to XCDs largest first, each to the least loaded one with a
  // free slot; the spare slots of an XCD then go one at a time to its matrix with the most
  // factor entries per group (at most GMAX, at least two blocks of rows per group).  If
  // there are more matrices than slots every matrix gets one group (no waits at all).
  int dev = 0, cus = 0, per_cu = 0;
  GX_HIP(hipGetDevice(&dev));
  GX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const void* kf = m.fp32 ? reinterpret_cast<const void*>(&k_band_solve_1_multi<float>)
                          : reinterpret_cast<const void*>(&k_band_solve_1_multi<double>);
  GX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, SOLVE_THREADS, 0));
  const int NX = cus % 8 == 0 ? 8 : 1;             // XCDs (MI355X: 8 of 32 CUs)
  const int64_t per_x = (int64_t)cus / NX * std::max(per_cu, 1);
  const int nm = m.n_mat;
  std::vector<int> xcd(nm, 0);
  std::vector<double> wk(nm);
  for (int j = 0; j < nm; ++j) {
    wk[j] = (double)m.host[j].n * (double)(m.host[j].B + 1);
    m.host[j].G = 1;
  }
  std::vector<int> order(nm);
  for (int j = 0; j < nm; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return wk[a] > wk[b]; });
  std::vector<double> load(NX, 0.0);
  std::vector<int64_t> used(NX, 0);
  const bool fits = nm <= per_x * NX;
  for (int r = 0; r < nm; ++r) {
    const int j = order[r];
    int best = -1;
    for (int x = 0; x < NX; ++x)
      if ((!fits || used[x] < per_x) && (best < 0 || load[x] < load[best])) best = x;
    xcd[j] = best;
    load[best] += wk[j];
    ++used[best];
  }
  if (fits)
    for (int x = 0; x < NX; ++x)
      for (; used[x] < per_x; ++used[x]) {
        int pick = -1;
        for (int j = 0; j < nm; ++j) {
          const BandPtrs& t = m.host[j];
          if (xcd[j] != x || t.G >= GMAX || t.n < (int64_t)2 * SB * (t.G + 1)) continue;
          if (pick < 0 || wk[j] / (double)t.G > wk[pick] / (double)m.host[pick].G) pick = j;
        }
        if (pick < 0) break;
        ++m.host[pick].G;
      }
  std::vector<std::vector<int32_t>> lists(NX);
  for (int j = 0; j < nm; ++j)
    for (int g = 0; g < (int)m.host[j].G; ++g) {
      lists[xcd[j]].push_back(j);
      lists[xcd[j]].push_back(g);
    }
  size_t slots = 0;
  for (auto& l : lists) slots = std::max(slots, l.size() / 2);
  std::vector<int32_t> wl(2 * slots * NX, -1);
  for (int x = 0; x < NX; ++x)
    for (size_t q = 0; q < lists[x].size() / 2; ++q) {
      wl[2 * (q * NX + x)] = lists[x][2 * q];
      wl[2 * (q * NX + x) + 1] = lists[x][2 * q + 1];
    }
  m.n_wg = (int)(slots * NX);
  if (m.tab.n < m.host.size()) m.tab.alloc(m.host.size());
  to_dev(m.tab.p, m.host.data(), m.host.size(), st);
  if (m.work.n < wl.size()) m.work.alloc(wl.size());
  to_dev(m.work.p, wl.data(), wl.size(), st);
  if (!m.err.n) {
    m.err.alloc(1);
    zero(m.err, st);
  }
  GX_HIP(hipStreamSynchronize(st));                // wl and host are read by the copies
}

// Solves every matrix of the table in place (marker fill, solve, copy-out on st).
void multi_solve(MultiSolve& m, hipStream_t st) {
  GX_REQUIRE(m.n_mat > 0, "multi-set solve: no table");
  const unsigned nm = (unsigned)m.n_mat;
  hipLaunchKernelGGL(k_fill_mark_multi, dim3(nblocks((m.max_n + SB - 1) / SB * SB, 256), nm),
                     dim3(256), 0, st, m.tab.p);
  if (m.fp32)
    hipLaunchKernelGGL(k_band_solve_1_multi<float>, dim3((unsigned)m.n_wg), dim3(SOLVE_THREADS),
                       0, st, m.tab.p, m.work.p, m.err.p);
  else
    hipLaunchKernelGGL(k_band_solve_1_multi<double>, dim3((unsigned)m.n_wg), dim3(SOLVE_THREADS),
                       0, st, m.tab.p, m.work.p, m.err.p);
  hipLaunchKernelGGL(k_copy_out_multi, dim3(nblocks(m.max_n, 256), nm), dim3(256), 0, st,
                     m.tab.p);
  GX_HIP(hipGetLastError());
}

// Raises if a multi-set solve since the last check timed out waiting for a block.
void multi_solve_check(MultiSolve& m, hipStream_t st) {
  if (!m.err.n) return;
  int h = 0;
  to_host(&h, m.err.p, 1, st);
  if (h) {
    zero(m.err, st);
    throw Error(GX_EHIP, "banded solve: a work-group timed out waiting for a block");
  }
}

// Raises if a multi-work-group solve since the last check timed out waiting for a block.
void band_solve_check(BandSet& bs, hipStream_t st) {
  if (!bs.err.n) return;
  int h = 0;
  to_host(&h, bs.err.p, 1, st);
  if (h) {
    zero(bs.err, st);
    throw Error(GX_EHIP, "banded solve: a work-group timed out waiting for a block");
  }
}

void band_layout(BandSet& bs, const std::vector<int64_t>& n, const std::vector<int64_t>& B,
                 bool fp32, hipStream_t st) {
  bs.n_mat = (int)n.size();
  bs.n = n;
  bs.B = B;
  bs.ld.resize(n.size());
  bs.off.resize(n.size());
  bs.fp32 = fp32;
  int64_t o = 0;
  bs.max_n = 0;
  bs.panel.release();
  bs.d_poff.release();
  bs.ybuf.release();
  bs.d_yoff.release();
  bs.mbuf.release();
  bs.max_B = 0;
  for (size_t j = 0; j < n.size(); ++j) {
    bs.ld[j] = B[j] + 1;
    bs.off[j] = o;
    o += n[j] * bs.ld[j];
    bs.max_n = std::max<int64_t>(bs.max_n, n[j]);
    bs.max_B = std::max<int64_t>(bs.max_B, B[j]);
  }
  bs.total = o;
  bs.env.assign(n.size(), 0);
  for (size_t j = 0; j < n.size(); ++j) {      // the band itself: row r holds min(r, B) + 1
    const int64_t m = std::min(n[j], B[j] + 1);
    bs.env[j] = m * (m + 1) / 2 + (n[j] - m) * (B[j] + 1);
  }
  bs.d_n.alloc(n.size());
  bs.d_B.alloc(n.size());
  bs.d_ld.alloc(n.size());
  bs.d_off.alloc(n.size());
  to_dev(bs.d_n.p, bs.n.data(), n.size(), st);
  to_dev(bs.d_B.p, bs.B.data(), n.size(), st);
  to_dev(bs.d_ld.p, bs.ld.data(), n.size(), st);
  to_dev(bs.d_off.p, bs.off.data(), n.size(), st);
  bs.boff.assign(n.size() + 1, 0);
  for (size_t j = 0; j < n.size(); ++j)
    bs.boff[j + 1] = bs.boff[j] + (n[j] + SB - 1) / SB * SB * SB;
  bs.d_boff.alloc(n.size() + 1);
  to_dev(bs.d_boff.p, bs.boff.data(), n.size() + 1, st);
  if (fp32) {
    bs.v64.release();
    bs.dinv64.release();
    bs.v32.alloc(o + BAND_PAD);
    GX_HIP(hipMemsetAsync(bs.v32.p + o, 0, BAND_PAD * sizeof(float), st));
    bs.dinv32.alloc(bs.boff[n.size()]);
  } else {
    bs.v32.release();
    bs.dinv32.release();
    bs.v64.alloc(o + BAND_PAD);
    GX_HIP(hipMemsetAsync(bs.v64.p + o, 0, BAND_PAD * sizeof(double), st));
    bs.dinv64.alloc(bs.boff[n.size()]);
  }
  bs.solve_groups[0] = bs.solve_groups[1] = 0;
  GX_HIP(hipStreamSynchronize(st));
}


// ---------------------------------------------------------------------------------------
// Stand-alone factor-and-solve of caller-supplied band matrices (exposed for testing the
// subdomain solver in isolation).
__global__ void k_band_import(int64_t total, const double* src, const double* dscale,
                              const int64_t* off, const int64_t* nn, const int64_t* bw,
                              const int64_t* doff, int n_mat, float* d32, double* d64) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int j = 0;
  while (j + 1 < n_mat && off[j + 1] <= e) ++j;
  const int64_t B = bw[j], r = (e - off[j]) / (B + 1), c = r + (e - off[j]) % (B + 1) - B;
  double v = src[e];
  if (dscale) v *= (c >= 0) ? dscale[doff[j] + r] * dscale[doff[j] + c] : 0.0;
  if (d32) d32[e] = (float)v;
  else d64[e] = v;
}

__global__ void k_band_diag(int64_t rows, const double* src, const int64_t* off,
                            const int64_t* nn, const int64_t* bw, const int64_t* doff, int n_mat,
                            double* dscale) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows) return;
  int j = 0;
  while (j + 1 < n_mat && doff[j + 1] <= q) ++j;
  const int64_t r = q - doff[j];
  const double d = src[off[j] + r * (bw[j] + 1) + bw[j]];
  dscale[q] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
}

__global__ void k_scale_rhs(int64_t rows, int nrhs, const double* dscale, double* x) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * nrhs) return;
  x[e] *= dscale[e / nrhs];
}

}  // namespace gx

extern "C" gx_status gx_band_factor_solve(gx_ctx* c, int32_t n_mat, const int64_t* n,
                                          const int64_t* bw, const double* band,
                                          int32_t precision, int32_t nrhs, int32_t groups,
                                          double* x) {
  using namespace gx;
  GX_API_BEGIN(c)
  GX_REQUIRE(n_mat >= 1 && n && bw && band && x, "bad band matrices");
  GX_REQUIRE(precision == GX_FP64 || precision == GX_MIXED, "bad precision");
  GX_REQUIRE(nrhs == 1 || (nrhs % 8 == 0 && nrhs <= 2 * MC),
             "nrhs must be 1 or a multiple of 8 up to 64");
  std::vector<int64_t> nv(n, n + n_mat), bv(bw, bw + n_mat), off(n_mat + 1, 0),
      doff(n_mat + 1, 0), xoff(n_mat);
  for (int j = 0; j < n_mat; ++j) {
    GX_REQUIRE(nv[j] >= 1 && bv[j] >= 0 && bv[j] < nv[j], "bad order or bandwidth");
    off[j + 1] = off[j] + nv[j] * (bv[j] + 1);
    doff[j + 1] = doff[j] + nv[j];
    xoff[j] = doff[j] * nrhs;
  }
  hipStream_t s = c->stream;
  const bool fp32 = precision == GX_MIXED;
  BandSet bs;
  band_layout(bs, nv, bv, fp32, s);
  bs.force_groups[0] = bs.force_groups[1] = groups;
  DevBuf<int64_t> d_off(n_mat + 1), d_doff(n_mat + 1), d_xoff(n_mat);
  to_dev(d_off.p, off.data(), n_mat + 1, s);
  to_dev(d_doff.p, doff.data(), n_mat + 1, s);
  to_dev(d_xoff.p, xoff.data(), n_mat, s);
  DevBuf<double> dsc;
  if (fp32) {
    dsc.alloc(doff[n_mat]);
    hipLaunchKernelGGL(k_band_diag, dim3(nblocks(doff[n_mat], 256)), dim3(256), 0, s,
                       doff[n_mat], band, d_off.p, bs.d_n.p, bs.d_B.p, d_doff.p, n_mat, dsc.p);
  }
  hipLaunchKernelGGL(k_band_import, dim3(nblocks(off[n_mat], 256)), dim3(256), 0, s,
                     off[n_mat], band, fp32 ? dsc.p : nullptr, d_off.p, bs.d_n.p, bs.d_B.p,
                     d_doff.p, n_mat, fp32 ? bs.v32.p : nullptr, fp32 ? nullptr : bs.v64.p);
  GX_HIP(hipGetLastError());
  band_factor(bs, s, "the given band matrices");
  if (fp32)
    hipLaunchKernelGGL(k_scale_rhs, dim3(nblocks(doff[n_mat] * nrhs, 256)), dim3(256), 0, s,
                       doff[n_mat], nrhs, dsc.p, x);
  band_solve(bs, d_xoff.p, x, s, nrhs);
  if (fp32)
    hipLaunchKernelGGL(k_scale_rhs, dim3(nblocks(doff[n_mat] * nrhs, 256)), dim3(256), 0, s,
                       doff[n_mat], nrhs, dsc.p, x);
  GX_HIP(hipGetLastError());
  band_solve_check(bs, s);
  GX_HIP(hipStreamSynchronize(s));
  GX_API_END(c)
}

namespace gx {

}  // namespace gx
