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

constexpr int NB = 32;          // factorisation block
constexpr int TS = 32;          // trailing-update tile
constexpr int SB = 64;          // solve block (one wavefront)
constexpr int WIN = 4096;       // solve window (power of two), holds B + SB values
constexpr int SOLVE_THREADS = 512;

struct BandArgs {
  const int64_t* n;
  const int64_t* B;
  const int64_t* ld;
  const int64_t* off;
};

template <class T>
__global__ void __launch_bounds__(256) k_potrf(BandArgs a, T* v, int64_t c0, int* err) {
  __shared__ double D[NB][NB + 1];
  const int j = blockIdx.x;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (c0 >= n) return;
  T* base = v + a.off[j];
  const int nb = (int)min<int64_t>(NB, n - c0);
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int i = idx / NB, l = idx % NB;
    double x = 0.0;
    if (i < nb && l <= i && i - l <= B) x = (double)base[(c0 + i) * ld + (l - i + B)];
    D[i][l] = x;
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
  for (int idx = threadIdx.x; idx < nb * nb; idx += blockDim.x) {
    const int i = idx / nb, l = idx % nb;
    if (l <= i && i - l <= B) base[(c0 + i) * ld + (l - i + B)] = (T)D[i][l];
  }
}

// panel rows r in [c0 + nb, c0 + nb + B): solve x L_kk^T = a for the row's entries in the
// block columns [c0, c0 + nb)
template <class T>
__global__ void __launch_bounds__(256) k_trsm(BandArgs a, T* v, int64_t c0) {
  __shared__ double L[NB][NB + 1];
  const int j = blockIdx.y;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (c0 >= n) return;
  const int nb = (int)min<int64_t>(NB, n - c0);
  const int64_t nrow = min<int64_t>(B, n - c0 - nb);
  if ((int64_t)blockIdx.x * blockDim.x >= nrow) return;
  T* base = v + a.off[j];
  for (int idx = threadIdx.x; idx < NB * NB; idx += blockDim.x) {
    const int i = idx / NB, l = idx % NB;
    double x = 0.0;
    if (i < nb && l <= i && i - l <= B) x = (double)base[(c0 + i) * ld + (l - i + B)];
    L[i][l] = x;
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrow) return;
  const int64_t r = c0 + nb + t;
  T* row = base + r * ld + (c0 - r + B);        // row[i] = entry (r, c0 + i), valid if >= 0
  const int64_t first = r - B - c0;              // entries i < first lie outside the band
  double x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    double s = (i < nb && i >= first) ? (double)row[i] : 0.0;
#pragma unroll
    for (int l = 0; l < i; ++l) s -= x[l] * L[i][l];
    x[i] = (i < nb) ? s / L[i][i] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < nb && i >= first) row[i] = (T)x[i];
}

// trailing update of rows/cols [c0 + nb, c0 + nb + W): A[r][s] -= sum_c L[r][c] L[s][c]
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
  for (int idx = threadIdx.x; idx < TS * NB; idx += blockDim.x) {
    const int i = idx / NB, c = idx % NB;
    const int64_t r = r0 + i, s = s0 + i, col = c0 + c;
    Pr[i][c] = (c < nb && r < wend && col >= r - B) ? (double)base[r * ld + (col - r + B)] : 0.0;
    Ps[i][c] = (c < nb && s < wend && col >= s - B) ? (double)base[s * ld + (col - s + B)] : 0.0;
  }
  __syncthreads();
  const int i = threadIdx.x / 8, l0 = (threadIdx.x % 8) * 4;
  double acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  for (int c = 0; c < NB; ++c) {
    const double p = Pr[i][c];
    acc0 += p * Ps[l0][c];
    acc1 += p * Ps[l0 + 1][c];
    acc2 += p * Ps[l0 + 2][c];
    acc3 += p * Ps[l0 + 3][c];
  }
  const int64_t r = r0 + i;
  if (r >= wend) return;
  const double acc[4] = {acc0, acc1, acc2, acc3};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t s = s0 + l0 + q;
    if (s <= r && s < wend) {
      T* e = base + r * ld + (s - r + B);
      *e = (T)((double)*e - acc[q]);
    }
  }
}

template <class T>
void band_factor_t(BandSet& bs, T* v, hipStream_t st, int* err) {
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p};
  const int64_t steps = (bs.max_n + NB - 1) / NB;
  const int64_t nt = (bs.max_B + TS - 1) / TS;
  const unsigned tiles = (unsigned)(nt * (nt + 1) / 2);
  const unsigned trsm_blocks = (unsigned)((bs.max_B + 255) / 256);
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t c0 = k * NB;
    hipLaunchKernelGGL(k_potrf<T>, dim3(bs.n_mat), dim3(256), 0, st, a, v, c0, err);
    if (bs.max_B > 0) {
      hipLaunchKernelGGL(k_trsm<T>, dim3(trsm_blocks, bs.n_mat), dim3(256), 0, st, a, v, c0);
      hipLaunchKernelGGL(k_syrk<T>, dim3(tiles, bs.n_mat), dim3(256), 0, st, a, v, c0);
    }
  }
  GX_HIP(hipGetLastError());
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
// Solves.  x (vector of matrix j at xoff[j]) is overwritten: forward then backward.

// Column blockIdx.y of matrix j's right-hand sides, stored with row stride `stride` at
// xoff[j] (stride 1 and one column for the preconditioner; row-major blocks of columns for
// the eigensolver).  Matrices with active[j] == 0 are skipped.
template <class T, class V>
__global__ void __launch_bounds__(SOLVE_THREADS) k_band_solve(BandArgs a, const T* v,
                                                             const int64_t* xoff, V* xall,
                                                             int stride,
                                                             const int32_t* active) {
  __shared__ double win[WIN];
  __shared__ double tri[SB][SB + 1];
  __shared__ double acc[SB];
  __shared__ double part[SOLVE_THREADS / 64][SB];
  const int j = blockIdx.x;
  if (active && !active[j]) return;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  const T* base = v + a.off[j];
  V* xv = xall + xoff[j] + blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#define x(i) xv[(int64_t)(i) * stride]
  constexpr int NW = SOLVE_THREADS / 64;
  constexpr int64_t MSK = WIN - 1;
  // ---- forward: L y = b
  for (int64_t i0 = 0; i0 < n; i0 += SB) {
    const int nb = (int)min<int64_t>(SB, n - i0);
    for (int ii = wave; ii < nb; ii += NW) {
      const int64_t i = i0 + ii;
      const T* row = base + i * ld + (B - i);    // row[c] = entry (i, c)
      const int64_t cs = max<int64_t>(i - B, 0);
      double s = 0.0;
      for (int64_t c = cs + lane; c < i0; c += 64) s += (double)row[c] * win[c & MSK];
      s = wave_sum_d(s);
      if (lane == 0) acc[ii] = (double)x(i) - s;
      for (int l = lane; l < SB; l += 64)
        tri[ii][l] = (l <= ii && i - (i0 + l) <= B) ? (double)row[i0 + l] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      double a_l = lane < nb ? acc[lane] : 0.0, y_l = 0.0;
      for (int c = 0; c < nb; ++c) {
        const double yc = __shfl(a_l, c) / tri[c][c];
        if (lane == c) y_l = yc;
        if (lane > c) a_l -= tri[lane][c] * yc;
      }
      if (lane < nb) {
        win[(i0 + lane) & MSK] = y_l;
        x(i0 + lane) = (V)y_l;
      }
    }
    __syncthreads();
  }
  // ---- backward: L^T x = y
  const int64_t nblk = (n + SB - 1) / SB;
  for (int64_t kb = nblk - 1; kb >= 0; --kb) {
    const int64_t i0 = kb * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t rend = min<int64_t>(n, i0 + nb + B);
    double s = 0.0;
    const int64_t c = i0 + lane;
    for (int64_t r = i0 + nb + wave; r < rend; r += NW)
      if (lane < nb && r - B <= c) s += (double)base[r * ld + (c - r + B)] * win[r & MSK];
    part[wave][lane] = s;
    for (int ii = wave; ii < nb; ii += NW) {
      const int64_t i = i0 + ii;
      const T* row = base + i * ld + (B - i);
      for (int l = lane; l < SB; l += 64)
        tri[ii][l] = (l <= ii && i - (i0 + l) <= B) ? (double)row[i0 + l] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += part[w][lane];
      double a_l = lane < nb ? (double)x(i0 + lane) - t : 0.0, x_l = 0.0;
      for (int cc = nb - 1; cc >= 0; --cc) {
        const double xc = __shfl(a_l, cc) / tri[cc][cc];
        if (lane == cc) x_l = xc;
        if (lane < cc) a_l -= tri[cc][lane] * xc;
      }
      if (lane < nb) {
        win[(i0 + lane) & MSK] = x_l;
        x(i0 + lane) = (V)x_l;
      }
    }
    __syncthreads();
  }
#undef x
}

void band_solve(BandSet& bs, const int64_t* d_xoff, double* x64, float* x32, hipStream_t st,
                int ncol, const int32_t* active) {
  GX_REQUIRE(bs.max_B + SB <= WIN, "band too wide for the solve window");
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p};
  if (bs.fp32 && x32)
    hipLaunchKernelGGL((k_band_solve<float, float>), dim3(bs.n_mat, ncol), dim3(SOLVE_THREADS),
                       0, st, a, bs.v32.p, d_xoff, x32, ncol, active);
  else if (bs.fp32)
    hipLaunchKernelGGL((k_band_solve<float, double>), dim3(bs.n_mat, ncol),
                       dim3(SOLVE_THREADS), 0, st, a, bs.v32.p, d_xoff, x64, ncol, active);
  else
    hipLaunchKernelGGL((k_band_solve<double, double>), dim3(bs.n_mat, ncol),
                       dim3(SOLVE_THREADS), 0, st, a, bs.v64.p, d_xoff, x64, ncol, active);
  GX_HIP(hipGetLastError());
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
