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
// diagonal block in LDS, one solves the panel rows, one updates the trailing window with
// 32x32 tiles.  Matrices of different size and bandwidth run in the same launches.
//
// Solves: one work-group per matrix streams the band once forward (L y = b) and once
// backward (L^T x = y); a ring buffer in LDS holds the last B solved values, the 64x64
// diagonal triangle of each block is solved by one wavefront with lane shuffles.
#include "gx_internal.h"

namespace gx {

constexpr int NB = 64;          // factorisation block
constexpr int TS = 64;          // trailing-update tile
constexpr int SB = 64;          // solve block (one wavefront)
constexpr int SOLVE_THREADS = 512;

struct BandArgs {
  const int64_t* n;
  const int64_t* B;
  const int64_t* ld;
  const int64_t* off;
};

// Diagonal block of step c0: Cholesky in LDS, written back; its inverse goes to inv[j].
template <class T>
__global__ void __launch_bounds__(256) k_potrf(BandArgs a, T* v, int64_t c0, double* inv,
                                               int* err) {
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
  for (int i = 0; i < nb; ++i) {
    if (threadIdx.x == 0) {
      double d = D[i][i];
      if (!(d > 0.0)) {
        atomicOr(err, 1);
        d = 1.0;
      }
      D[i][i] = sqrt(d);
    }
    __syncthreads();
    for (int r = i + 1 + threadIdx.x; r < nb; r += blockDim.x) D[r][i] /= D[i][i];
    __syncthreads();
    const int m = nb - i - 1;
    for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) {
      const int r = i + 1 + idx / m, s = i + 1 + idx % m;
      if (s <= r) D[r][s] -= D[r][i] * D[s][i];
    }
    __syncthreads();
  }
  // inverse of the lower triangle, one column per thread (padding rows are identity)
  if (threadIdx.x < NB) {
    const int c = threadIdx.x;
    for (int i = 0; i < NB; ++i) {
      double sum = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) sum -= D[i][k] * Li[k][c];
      Li[i][c] = (i < c) ? 0.0 : sum / D[i][i];
    }
  }
  __syncthreads();
  double* ij = inv + (int64_t)j * NB * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int i = idx / NB, l = idx % NB;
    ij[idx] = Li[i][l];
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

// trailing update of rows/cols [c0 + nb, c0 + nb + W): A[r][s] -= sum_c L[r][c] L[s][c],
// 64x64 tiles of the lower triangle, 4x4 outputs per thread
template <class T>
__global__ void __launch_bounds__(256) k_syrk(BandArgs a, T* v, int64_t c0) {
  __shared__ double Pr[TS][NB + 1], Ps[TS][NB + 1];
  const int j = blockIdx.y;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (c0 >= n) return;
  const int nb = (int)min<int64_t>(NB, n - c0);
  const int64_t W = min<int64_t>(B, n - c0 - nb);
  if (W <= 0) return;
  const int64_t nt = (W + TS - 1) / TS;
  const int64_t tile = blockIdx.x;
  if (tile >= nt * (nt + 1) / 2) return;
  int64_t tr = 0, rem = tile;                    // lower-triangular tile enumeration
  while (rem > tr) { rem -= tr + 1; ++tr; }
  const int64_t ts = rem;
  T* base = v + a.off[j];
  const int64_t r0 = c0 + nb + tr * TS, s0 = c0 + nb + ts * TS, wend = c0 + nb + W;
  {
    constexpr int L = TS * NB / 256;             // 16 + 16 loads per thread, issued together
    double vr[L], vs[L];
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int idx = threadIdx.x + 256 * u;
      const int i = idx / NB, c = idx % NB;
      const int64_t r = r0 + i, ss = s0 + i, col = c0 + c;
      vr[u] = (c < nb && r < wend && col >= r - B) ? (double)base[r * ld + (col - r + B)] : 0.0;
      vs[u] = (c < nb && ss < wend && col >= ss - B) ? (double)base[ss * ld + (col - ss + B)] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < L; ++u) {
      const int idx = threadIdx.x + 256 * u;
      Pr[idx / NB][idx % NB] = vr[u];
      Ps[idx / NB][idx % NB] = vs[u];
    }
  }
  __syncthreads();
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int c = 0; c < NB; ++c) {
    double pr[4], ps[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) pr[p] = Pr[4 * ty + p][c];
#pragma unroll
    for (int q = 0; q < 4; ++q) ps[q] = Ps[4 * tx + q][c];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[p][q] += pr[p] * ps[q];
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t r = r0 + 4 * ty + p;
    if (r >= wend) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t s = s0 + 4 * tx + q;
      if (s <= r && s < wend) {
        T* e = base + r * ld + (s - r + B);
        *e = (T)((double)*e - acc[p][q]);
      }
    }
  }
}

template <class T>
void band_factor_t(BandSet& bs, T* v, hipStream_t st, int* err) {
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p};
  DevBuf<double> inv((size_t)bs.n_mat * NB * NB);
  const int64_t steps = (bs.max_n + NB - 1) / NB;
  const int64_t nt = (bs.max_B + TS - 1) / TS;
  const unsigned tiles = (unsigned)(nt * (nt + 1) / 2);
  const unsigned trsm_blocks = (unsigned)((bs.max_B + TS - 1) / TS);
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t c0 = k * NB;
    hipLaunchKernelGGL(k_potrf<T>, dim3(bs.n_mat), dim3(256), 0, st, a, v, c0, inv.p, err);
    if (bs.max_B > 0) {
      hipLaunchKernelGGL(k_trsm<T>, dim3(trsm_blocks, bs.n_mat), dim3(256), 0, st, a, v, c0,
                         inv.p);
      hipLaunchKernelGGL(k_syrk<T>, dim3(tiles, bs.n_mat), dim3(256), 0, st, a, v, c0);
    }
  }
  GX_HIP(hipGetLastError());
  GX_HIP(hipStreamSynchronize(st));
}

void band_factor(BandSet& bs, hipStream_t st) {
  DevBuf<int> err(1);
  zero(err, st);
  if (bs.fp32)
    band_factor_t<float>(bs, bs.v32.p, st, err.p);
  else
    band_factor_t<double>(bs, bs.v64.p, st, err.p);
  int h = 0;
  to_host(&h, err.p, 1, st);
  if (h) throw Error(GX_ENOTSPD, "non-positive pivot in a banded Cholesky factorisation");
}

// ---------------------------------------------------------------------------------------
// Solves.  NC right-hand-side columns per work-group, stored row-major with row stride
// `stride` at xoff[j] (+ NC * blockIdx.y); overwritten: forward (L y = b), then backward
// (L^T x = y).  8 wavefronts: in the forward dot phase wave w owns rows 8w..8w+7 of the
// 64-row block, so every loaded solution value serves 8 band rows; in the backward phase
// lanes own the block's 64 columns and waves split the band rows below it; the 64x64
// diagonal triangle of each block is solved per column by one wave with lane shuffles.
// Solution values written earlier by the work-group are read back through global memory
// (same work-group, ordered by the barriers).
constexpr int SW = SOLVE_THREADS / 64;           // waves per work-group (8)
constexpr int RPW = SB / SW;                      // forward rows per wave (8)

// the 64x64 diagonal triangle of a solve block into LDS (rows 8w..8w+7 per wave; all
// loads issued before the stores); rows past the end of the matrix become identity
template <class T>
__device__ inline void load_tri(double (&tri)[SB][SB + 1], const T* base, int64_t B,
                                int64_t ld, int64_t i0, int nb, int lane, int wave) {
  double v[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int ii = RPW * wave + r;
    const int64_t i = i0 + ii;
    v[r] = (ii < nb && lane <= ii && i - (i0 + lane) <= B)
               ? (double)base[i * ld + (i0 + lane - i + B)]
               : (lane == ii ? 1.0 : 0.0);
  }
#pragma unroll
  for (int r = 0; r < RPW; ++r) tri[RPW * wave + r][lane] = v[r];
}

template <class T, class V, int NC>
__global__ void __launch_bounds__(SOLVE_THREADS) k_band_solve(BandArgs a, const T* v,
                                                             const int64_t* xoff, V* xall,
                                                             int stride, int ncol,
                                                             const int32_t* active) {
  __shared__ double tri[SB][SB + 1];
  __shared__ double acc[SB][NC];
  __shared__ double part[SW][SB][NC];
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  const int col0 = blockIdx.y * NC;
  const int nc = min(NC, ncol - col0);
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  const T* base = v + a.off[j];
  V* xv = xall + xoff[j] + col0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#define X(i, c) xv[(int64_t)(i) * stride + (c)]
  // ---- forward: L y = b
  for (int64_t i0 = 0; i0 < n; i0 += SB) {
    const int nb = (int)min<int64_t>(SB, n - i0);
    constexpr int RH = NC == 1 ? RPW : 4;           // rows accumulated per pass
    for (int h = 0; h < RPW / RH; ++h) {
      const int64_t ifirst = i0 + RPW * wave + RH * h;
      double s[RH][NC];
#pragma unroll
      for (int r = 0; r < RH; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) s[r][c] = 0.0;
      if (ifirst < n) {
        for (int64_t cc = max<int64_t>(ifirst - B, 0) + lane; cc < i0; cc += 64) {
          double y[NC];
#pragma unroll
          for (int c = 0; c < NC; ++c) y[c] = c < nc ? (double)X(cc, c) : 0.0;
#pragma unroll
          for (int r = 0; r < RH; ++r) {
            const int64_t i = ifirst + r;
            const double l =
                (i < n && cc >= i - B) ? (double)base[i * ld + (cc - i + B)] : 0.0;
#pragma unroll
            for (int c = 0; c < NC; ++c) s[r][c] += l * y[c];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RH; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) s[r][c] = wave_sum_d(s[r][c]);
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < RH; ++r) {
          const int64_t i = ifirst + r;
#pragma unroll
          for (int c = 0; c < NC; ++c)
            acc[RPW * wave + RH * h + r][c] = (i < n && c < nc) ? (double)X(i, c) - s[r][c] : 0.0;
        }
      }
    }
    load_tri<T>(tri, base, B, ld, i0, nb, lane, wave);
    __syncthreads();
    if (wave < nc) {
      double a_l = acc[lane][wave], y_l = 0.0;
      for (int k = 0; k < nb; ++k) {
        const double yk = __shfl(a_l, k) / tri[k][k];
        if (lane == k) y_l = yk;
        if (lane > k) a_l -= tri[lane][k] * yk;
      }
      if (lane < nb) X(i0 + lane, wave) = (V)y_l;
    }
    __syncthreads();
  }
  // ---- backward: L^T x = y
  const int64_t nblk = (n + SB - 1) / SB;
  for (int64_t kb = nblk - 1; kb >= 0; --kb) {
    const int64_t i0 = kb * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t rend = min<int64_t>(n, i0 + nb + B);
    const int64_t cidx = i0 + lane;
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) s[c] = 0.0;
    int64_t r = i0 + nb + wave;
    constexpr int UB = NC == 1 ? 4 : 1;           // rows in flight per lane
    if (UB > 1) {
      for (; r + (UB - 1) * SW < rend; r += UB * SW) {
        double l[UB], xr[UB][NC];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int64_t rr = r + u * SW;
          l[u] = (lane < nb && rr - B <= cidx) ? (double)base[rr * ld + (cidx - rr + B)] : 0.0;
#pragma unroll
          for (int c = 0; c < NC; ++c) xr[u][c] = c < nc ? (double)X(rr, c) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UB; ++u)
#pragma unroll
          for (int c = 0; c < NC; ++c) s[c] += l[u] * xr[u][c];
      }
    }
    for (; r < rend; r += SW) {
      const double l = (lane < nb && r - B <= cidx) ? (double)base[r * ld + (cidx - r + B)] : 0.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) s[c] += l * (c < nc ? (double)X(r, c) : 0.0);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) part[wave][lane][c] = s[c];
    load_tri<T>(tri, base, B, ld, i0, nb, lane, wave);
    __syncthreads();
    if (wave < nc) {
      double t = 0.0;
      for (int w = 0; w < SW; ++w) t += part[w][lane][wave];
      double a_l = lane < nb ? (double)X(i0 + lane, wave) - t : 0.0, x_l = 0.0;
      for (int k = nb - 1; k >= 0; --k) {
        const double xk = __shfl(a_l, k) / tri[k][k];
        if (lane == k) x_l = xk;
        if (lane < k) a_l -= tri[k][lane] * xk;
      }
      if (lane < nb) X(i0 + lane, wave) = (V)x_l;
    }
    __syncthreads();
  }
#undef X
}

// ---------------------------------------------------------------------------------------
// One right-hand side per matrix, G work-groups per matrix.  Block k of 64 rows belongs to
// work-group k mod G (forward) / (nblk - 1 - k) mod G (backward).  A work-group first adds
// the contributions of blocks that are complete by construction (its own previous block
// and everything before it), then waits - bounded spin, acquire - for the at most G - 1
// blocks still in flight, solves its diagonal triangle and publishes the block with a
// release store of the launch epoch.  A timed-out wait raises err and proceeds, so every
// wave always reaches the end of the kernel.
constexpr int64_t SPIN_LIMIT = (int64_t)1 << 24;

__device__ inline void wait_flag(const int* f, int epoch, int* err) {
  if (threadIdx.x == 0) {
    int64_t spins = 0;
    while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      if (++spins > SPIN_LIMIT) {
        atomicOr(err, 2);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

__device__ inline void post_flag(int* f, int epoch) {
  __hip_atomic_store(f, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T, class V>
__global__ void __launch_bounds__(SOLVE_THREADS) k_band_solve_mw(
    BandArgs a, const T* v, const int64_t* xoff, V* xall, int G, int n_pad, int n_mat,
    int* fflag, int* bflag, int64_t nblk_max, int epoch, int* err) {
  __shared__ double tri[SB][SB + 1];
  __shared__ double acc[SB];
  __shared__ double part[SW][SB];
  const int g = blockIdx.x / n_pad, j = blockIdx.x % n_pad;
  if (j >= n_mat || g >= G) return;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (n == 0) return;
  const T* base = v + a.off[j];
  V* x = xall + xoff[j];
  int* ff = fflag + (int64_t)j * nblk_max;
  int* bf = bflag + (int64_t)j * nblk_max;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nblk = (n + SB - 1) / SB;
  // ---- forward
  for (int64_t k = g; k < nblk; k += G) {
    const int64_t i0 = k * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t done_end = max<int64_t>(k - G + 1, 0) * SB;   // columns known complete
    const int64_t ifirst = i0 + RPW * wave;
    double s[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) s[r] = 0.0;
    for (int64_t cc = max<int64_t>(ifirst - B, 0) + lane; cc < done_end; cc += 64) {
      const double y = (double)x[cc];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int64_t i = ifirst + r;
        const double l = (i < n && cc >= i - B) ? (double)base[i * ld + (cc - i + B)] : 0.0;
        s[r] += l * y;
      }
    }
    load_tri<T>(tri, base, B, ld, i0, nb, lane, wave);
    for (int64_t kk = max<int64_t>(k - G + 1, 0); kk < k; ++kk) {   // blocks in flight
      wait_flag(ff + kk, epoch, err);
      const int64_t cc = kk * SB + lane;
      const double y = (double)x[cc];
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int64_t i = ifirst + r;
        const double l = (i < n && cc >= i - B) ? (double)base[i * ld + (cc - i + B)] : 0.0;
        s[r] += l * y;
      }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) s[r] = wave_sum_d(s[r]);
    if (lane == 0)
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const int64_t i = ifirst + r;
        acc[RPW * wave + r] = i < n ? (double)x[i] - s[r] : 0.0;
      }
    __syncthreads();
    if (wave == 0) {
      double a_l = acc[lane], y_l = 0.0;
      for (int q = 0; q < nb; ++q) {
        const double yq = __shfl(a_l, q) / tri[q][q];
        if (lane == q) y_l = yq;
        if (lane > q) a_l -= tri[lane][q] * yq;
      }
      if (lane < nb) x[i0 + lane] = (V)y_l;
      if (lane == 0) post_flag(ff + k, epoch);
    }
    __syncthreads();
  }
  // ---- backward
  for (int64_t t = g; t < nblk; t += G) {
    const int64_t kb = nblk - 1 - t;
    const int64_t i0 = kb * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t rend = min<int64_t>(n, i0 + nb + B);
    const int64_t inflight_end = min<int64_t>(rend, (kb + G) * SB);   // rows of blocks in flight
    const int64_t cidx = i0 + lane;
    wait_flag(ff + kb, epoch, err);                 // this block's forward result
    double sacc = 0.0;
    int64_t r = inflight_end + wave;
    for (; r + 3 * SW < rend; r += 4 * SW) {
      double l[4], xr[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t rr = r + u * SW;
        l[u] = (lane < nb && rr - B <= cidx) ? (double)base[rr * ld + (cidx - rr + B)] : 0.0;
        xr[u] = (double)x[rr];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) sacc += l[u] * xr[u];
    }
    for (; r < rend; r += SW) {
      const double l = (lane < nb && r - B <= cidx) ? (double)base[r * ld + (cidx - r + B)] : 0.0;
      sacc += l * (double)x[r];
    }
    load_tri<T>(tri, base, B, ld, i0, nb, lane, wave);
    for (int64_t kk = kb + 1; kk < min<int64_t>(kb + G, nblk); ++kk) {   // in flight
      wait_flag(bf + kk, epoch, err);
      for (int64_t rr = kk * SB + wave; rr < min<int64_t>((kk + 1) * SB, rend); rr += SW) {
        const double l = (lane < nb && rr - B <= cidx) ? (double)base[rr * ld + (cidx - rr + B)] : 0.0;
        sacc += l * (double)x[rr];
      }
    }
    part[wave][lane] = sacc;
    __syncthreads();
    if (wave == 0) {
      double tsum = 0.0;
      for (int w = 0; w < SW; ++w) tsum += part[w][lane];
      double a_l = lane < nb ? (double)x[i0 + lane] - tsum : 0.0, x_l = 0.0;
      for (int q = nb - 1; q >= 0; --q) {
        const double xq = __shfl(a_l, q) / tri[q][q];
        if (lane == q) x_l = xq;
        if (lane < q) a_l -= tri[q][lane] * xq;
      }
      if (lane < nb) x[i0 + lane] = (V)x_l;
      if (lane == 0) post_flag(bf + kb, epoch);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// m right-hand sides per matrix (m <= 64, row-major, row stride m), G work-groups per matrix
// pipelined as in k_band_solve_mw.  The dot products of a 64-row block are a
// (64 x B) x (B x m) product staged through LDS in 64-column chunks of the band; each
// thread accumulates 4 rows x 2 columns.  Triangles are solved per column by the waves.
constexpr int MC = 40;                           // right-hand-side columns per launch, max

template <class T>
__device__ inline void mc_chunk_fwd(double (&Ab)[SB][SB + 1], double (&Yc)[SB][MC + 1],
                                    const T* base, const double* x, int64_t n, int64_t B,
                                    int64_t ld, int64_t i0, int64_t c0, int64_t cend, int m) {
  // band rows i0..i0+63, columns c0..c0+63 (masked to the band, < cend); Y rows c0..c0+63.
  // All loads of a thread are issued before any LDS store (one memory round trip).
  constexpr int LA = SB * SB / SOLVE_THREADS;            // 8
  constexpr int LY = (SB * MC + SOLVE_THREADS - 1) / SOLVE_THREADS;   // 5
  double va[LA], vy[LY];
#pragma unroll
  for (int u = 0; u < LA; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    const int ii = idx / SB, kk = idx % SB;
    const int64_t i = i0 + ii, c = c0 + kk;
    va[u] = (i < n && c < cend && c >= i - B) ? (double)base[i * ld + (c - i + B)] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < LY; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    const int kk = idx / m, cc = idx - kk * m;
    const int64_t c = c0 + kk;
    vy[u] = (idx < SB * m && c < cend) ? x[c * m + cc] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < LA; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    Ab[idx / SB][idx % SB] = va[u];
  }
#pragma unroll
  for (int u = 0; u < LY; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    if (idx < SB * m) Yc[idx / m][idx - (idx / m) * m] = vy[u];
  }
  if (threadIdx.x < SB) Yc[threadIdx.x][MC] = 0.0;
}

// backward chunk: Ab[rr][cl] = L[r0 + rr][i0 + cl], Yc[rr][col] = x[r0 + rr][col]
template <class T>
__device__ inline void mc_chunk_bwd(double (&Ab)[SB][SB + 1], double (&Yc)[SB][MC + 1],
                                    const T* base, const double* x, int64_t B, int64_t ld,
                                    int64_t i0, int nb, int64_t r0, int64_t rr_end, int m) {
  constexpr int LA = SB * SB / SOLVE_THREADS;
  constexpr int LY = (SB * MC + SOLVE_THREADS - 1) / SOLVE_THREADS;
  double va[LA], vy[LY];
#pragma unroll
  for (int u = 0; u < LA; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    const int rr = idx / SB, cl = idx % SB;
    const int64_t r = r0 + rr, c = i0 + cl;
    va[u] = (r < rr_end && cl < nb && r - B <= c) ? (double)base[r * ld + (c - r + B)] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < LY; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    const int rr = idx / m, cc = idx - rr * m;
    const int64_t r = r0 + rr;
    vy[u] = (idx < SB * m && r < rr_end) ? x[r * m + cc] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < LA; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    Ab[idx / SB][idx % SB] = va[u];
  }
#pragma unroll
  for (int u = 0; u < LY; ++u) {
    const int idx = threadIdx.x + u * SOLVE_THREADS;
    if (idx < SB * m) Yc[idx / m][idx - (idx / m) * m] = vy[u];
  }
  if (threadIdx.x < SB) Yc[threadIdx.x][MC] = 0.0;
}

template <class T>
__global__ void __launch_bounds__(SOLVE_THREADS) k_band_solve_mc(
    BandArgs a, const T* v, const int64_t* xoff, double* xall, int m, int G, int n_pad,
    int n_mat, int* fflag, int* bflag, int64_t nblk_max, int epoch, const int32_t* active,
    int* err) {
  __shared__ double Ab[SB][SB + 1];               // band chunk; the block's triangle later
  __shared__ double Yc[SB][MC + 1];               // solution chunk
  __shared__ double acc[SB][MC + 1];
  double (&tri)[SB][SB + 1] = Ab;
  const int g = blockIdx.x / n_pad, j = blockIdx.x % n_pad;
  if (j >= n_mat || g >= G) return;
  if (active && !active[j]) return;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  const T* base = v + a.off[j];
  double* x = xall + xoff[j];
  int* ff = fflag + (int64_t)j * nblk_max;
  int* bf = bflag + (int64_t)j * nblk_max;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rg = threadIdx.x / 32, slot = threadIdx.x % 32;   // 16 row groups x 32 slots
  const int slot2 = slot + 32 < MC ? slot + 32 : MC;          // second column (MC: unused)
  const int64_t nblk = (n + SB - 1) / SB;
  // ---- forward
  for (int64_t k = g; k < nblk; k += G) {
    const int64_t i0 = k * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    double s[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    const int64_t cfirst = max<int64_t>(i0 - B, 0);
    const int64_t done_end = max<int64_t>(k - G + 1, 0) * SB;
    for (int64_t c0 = cfirst; c0 < i0; c0 += SB) {
      const int64_t kk = c0 / SB;                       // not block aligned at the start
      const int64_t cend = min<int64_t>(i0, c0 + SB);
      if (cend > done_end) {                            // part of a block still in flight
        const int64_t b0 = max<int64_t>(c0 / SB, done_end / SB);
        for (int64_t w = b0; w * SB < cend; ++w) wait_flag(ff + w, epoch, err);
      }
      (void)kk;
      mc_chunk_fwd<T>(Ab, Yc, base, x, n, B, ld, i0, c0, cend, m);
      __syncthreads();
      for (int q = 0; q < SB; ++q) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const double av = Ab[4 * rg + p][q];
          s[p][0] += av * Yc[q][slot];
          s[p][1] += av * Yc[q][slot2];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int ii = 4 * rg + p;
      const int64_t i = i0 + ii;
      if (slot < m) acc[ii][slot] = i < n ? x[i * m + slot] - s[p][0] : 0.0;
      if (slot + 32 < m) acc[ii][slot + 32] = i < n ? x[i * m + slot + 32] - s[p][1] : 0.0;
    }
    load_tri<T>(tri, base, B, ld, i0, nb, lane, wave);
    __syncthreads();
    for (int col = wave; col < m; col += SW) {
      double a_l = acc[lane][col], y_l = 0.0;
      for (int q = 0; q < nb; ++q) {
        const double yq = __shfl(a_l, q) / tri[q][q];
        if (lane == q) y_l = yq;
        if (lane > q) a_l -= tri[lane][q] * yq;
      }
      if (lane < nb) x[(i0 + lane) * m + col] = y_l;
    }
    __syncthreads();
    if (threadIdx.x == 0) post_flag(ff + k, epoch);
  }
  // ---- backward
  for (int64_t t = g; t < nblk; t += G) {
    const int64_t kb = nblk - 1 - t;
    const int64_t i0 = kb * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t rend = min<int64_t>(n, i0 + nb + B);
    const int64_t done_beg = min<int64_t>(n, (kb + G) * SB);   // rows known complete
    wait_flag(ff + kb, epoch, err);
    double s[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    // chunks of 64 rows from the far end of the band inwards: rows of complete blocks
    // first, the rows of blocks still in flight (right below this block) last
    const int64_t nchunk = (rend - (i0 + nb) + SB - 1) / SB;
    for (int64_t ch = nchunk - 1; ch >= 0; --ch) {
      const int64_t r0 = i0 + nb + ch * SB;
      const int64_t rr_end = min<int64_t>(rend, r0 + SB);
      if (r0 < done_beg)                                // rows of blocks still in flight
        for (int64_t w = r0 / SB; w * SB < min<int64_t>(rr_end, done_beg); ++w)
          wait_flag(bf + w, epoch, err);
      mc_chunk_bwd<T>(Ab, Yc, base, x, B, ld, i0, nb, r0, rr_end, m);
      __syncthreads();
      for (int q = 0; q < SB; ++q) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          const double av = Ab[q][4 * rg + p];
          s[p][0] += av * Yc[q][slot];
          s[p][1] += av * Yc[q][slot2];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int cl = 4 * rg + p;
      const int64_t c = i0 + cl;
      if (slot < m) acc[cl][slot] = cl < nb ? x[c * m + slot] - s[p][0] : 0.0;
      if (slot + 32 < m) acc[cl][slot + 32] = cl < nb ? x[c * m + slot + 32] - s[p][1] : 0.0;
    }
    load_tri<T>(tri, base, B, ld, i0, nb, lane, wave);
    __syncthreads();
    for (int col = wave; col < m; col += SW) {
      double a_l = acc[lane][col], x_l = 0.0;
      for (int q = nb - 1; q >= 0; --q) {
        const double xq = __shfl(a_l, q) / tri[q][q];
        if (lane == q) x_l = xq;
        if (lane < q) a_l -= tri[q][lane] * xq;
      }
      if (lane < nb) x[(i0 + lane) * m + col] = x_l;
    }
    __syncthreads();
    if (threadIdx.x == 0) post_flag(bf + kb, epoch);
  }
}

// Work-groups per matrix for the single right-hand-side solve: as many as keep every
// work-group of the launch resident at once (the waits rely on it), at most 4.
static int solve_groups(BandSet& bs, const void* kernel, int which) {
  if (bs.solve_groups[which] > 0) return bs.solve_groups[which];
  int dev = 0, cus = 0, per_cu = 0;
  GX_HIP(hipGetDevice(&dev));
  GX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  GX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, SOLVE_THREADS, 0));
  // the waits need every work-group of the launch resident: keep a quarter in reserve
  const int64_t capacity = (int64_t)cus * std::max(per_cu, 0) * 3 / 4;
  int G = 1;
  const int top = bs.force_groups[which] > 0 ? std::min(bs.force_groups[which], 8) : 4;
  for (int c = top; c >= 2; --c)
    if ((int64_t)bs.n_mat * c <= capacity && bs.max_n >= (int64_t)4 * SB * c) {
      G = c;
      break;
    }
  bs.solve_groups[which] = G;
  return G;
}

void band_solve(BandSet& bs, const int64_t* d_xoff, double* x64, float* x32, hipStream_t st,
                int ncol, const int32_t* active) {
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p};
  if (ncol == 1 && !active && !(bs.fp32 && x32)) {
    const int G = bs.fp32 ? solve_groups(bs, reinterpret_cast<const void*>(
                                                 &k_band_solve_mw<float, double>), 0)
                          : solve_groups(bs, reinterpret_cast<const void*>(
                                                 &k_band_solve_mw<double, double>), 0);
    if (G > 1) {
      const int64_t nblk = (bs.max_n + SB - 1) / SB;
      const int n_pad = (bs.n_mat + 7) / 8 * 8;
      if (bs.flags.n != (size_t)(2 * n_pad * nblk + 1)) {
        bs.flags.alloc(2 * n_pad * nblk + 1);
        zero(bs.flags, st);
        bs.epoch = 0;
      }
      ++bs.epoch;
      int* fl = bs.flags.p;
      if (bs.fp32)
        hipLaunchKernelGGL((k_band_solve_mw<float, double>), dim3(G * n_pad), dim3(SOLVE_THREADS),
                           0, st, a, bs.v32.p, d_xoff, x64, G, n_pad, bs.n_mat, fl,
                           fl + n_pad * nblk,
                           nblk, bs.epoch, fl + 2 * n_pad * nblk);
      else
        hipLaunchKernelGGL((k_band_solve_mw<double, double>), dim3(G * n_pad),
                           dim3(SOLVE_THREADS), 0, st, a, bs.v64.p, d_xoff, x64, G, n_pad,
                           bs.n_mat, fl, fl + n_pad * nblk, nblk, bs.epoch,
                           fl + 2 * n_pad * nblk);
      GX_HIP(hipGetLastError());
      return;
    }
  }
  if (ncol == 1) {
    const dim3 g(bs.n_mat, 1);
    if (bs.fp32 && x32)
      hipLaunchKernelGGL((k_band_solve<float, float, 1>), g, dim3(SOLVE_THREADS), 0, st, a,
                         bs.v32.p, d_xoff, x32, 1, 1, active);
    else if (bs.fp32)
      hipLaunchKernelGGL((k_band_solve<float, double, 1>), g, dim3(SOLVE_THREADS), 0, st, a,
                         bs.v32.p, d_xoff, x64, 1, 1, active);
    else
      hipLaunchKernelGGL((k_band_solve<double, double, 1>), g, dim3(SOLVE_THREADS), 0, st, a,
                         bs.v64.p, d_xoff, x64, 1, 1, active);
  } else if (ncol <= MC) {
    const int G = bs.fp32 ? solve_groups(bs, reinterpret_cast<const void*>(
                                                 &k_band_solve_mc<float>), 1)
                          : solve_groups(bs, reinterpret_cast<const void*>(
                                                 &k_band_solve_mc<double>), 1);
    const int64_t nblk = (bs.max_n + SB - 1) / SB;
    const int n_pad = (bs.n_mat + 7) / 8 * 8;
    if (bs.flags.n != (size_t)(2 * n_pad * nblk + 1)) {
      bs.flags.alloc(2 * n_pad * nblk + 1);
      zero(bs.flags, st);
      bs.epoch = 0;
    }
    ++bs.epoch;
    int* fl = bs.flags.p;
    if (bs.fp32)
      hipLaunchKernelGGL((k_band_solve_mc<float>), dim3(G * n_pad), dim3(SOLVE_THREADS), 0, st,
                         a, bs.v32.p, d_xoff, x64, ncol, G, n_pad, bs.n_mat, fl,
                         fl + n_pad * nblk, nblk, bs.epoch, active, fl + 2 * n_pad * nblk);
    else
      hipLaunchKernelGGL((k_band_solve_mc<double>), dim3(G * n_pad), dim3(SOLVE_THREADS), 0, st,
                         a, bs.v64.p, d_xoff, x64, ncol, G, n_pad, bs.n_mat, fl,
                         fl + n_pad * nblk, nblk, bs.epoch, active, fl + 2 * n_pad * nblk);
  } else {
    const dim3 g(bs.n_mat, (ncol + 7) / 8);
    if (bs.fp32)
      hipLaunchKernelGGL((k_band_solve<float, double, 8>), g, dim3(SOLVE_THREADS), 0, st, a,
                         bs.v32.p, d_xoff, x64, ncol, ncol, active);
    else
      hipLaunchKernelGGL((k_band_solve<double, double, 8>), g, dim3(SOLVE_THREADS), 0, st, a,
                         bs.v64.p, d_xoff, x64, ncol, ncol, active);
  }
  GX_HIP(hipGetLastError());
}

// Raises if a multi-work-group solve since the last check timed out waiting for a block.
void band_solve_check(BandSet& bs, hipStream_t st) {
  if (!bs.flags.n) return;
  int h = 0;
  to_host(&h, bs.flags.p + bs.flags.n - 1, 1, st);
  if (h) {
    zero(bs.flags, st);
    bs.epoch = 0;
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
  bs.max_B = 0;
  for (size_t j = 0; j < n.size(); ++j) {
    bs.ld[j] = B[j] + 1;
    bs.off[j] = o;
    o += n[j] * bs.ld[j];
    bs.max_n = std::max<int64_t>(bs.max_n, n[j]);
    bs.max_B = std::max<int64_t>(bs.max_B, B[j]);
  }
  bs.total = o;
  bs.d_n.alloc(n.size());
  bs.d_B.alloc(n.size());
  bs.d_ld.alloc(n.size());
  bs.d_off.alloc(n.size());
  to_dev(bs.d_n.p, bs.n.data(), n.size(), st);
  to_dev(bs.d_B.p, bs.B.data(), n.size(), st);
  to_dev(bs.d_ld.p, bs.ld.data(), n.size(), st);
  to_dev(bs.d_off.p, bs.off.data(), n.size(), st);
  if (fp32) {
    bs.v64.release();
    bs.v32.alloc(o);
  } else {
    bs.v32.release();
    bs.v64.alloc(o);
  }
  GX_HIP(hipStreamSynchronize(st));
}

}  // namespace gx
