// GenEO coarse space (section 2.3) and the setup entry point of the preconditioner.
//
// In every subdomain j the lowest-energy modes of the local generalised eigenproblem
//     A_j^N p = lambda X_j A_j^o X_j p
// are computed (A^N: stiffness of the subdomain's elements on all DOFs of its nodes;
// A^o: the same over the elements that also lie in another subdomain; X_j: partition of
// unity, zero off the interior).  Their partition-of-unity images span the coarse space;
// K_0 = Z^T K Z is factored once and solved in every preconditioner application.
//
// Eigensolver: block shift-invert subspace iteration with Rayleigh-Ritz for the largest
// mu of B p = mu M p, M = A^N + sigma B (lambda = 1/mu - sigma).  M is assembled in band
// storage directly from the element matrices and factored by the batched band Cholesky;
// B products are gathers over the stored element matrices of the overlap elements.
// With Y = M^-1 B X the M-products come for free (M Y = B X), so each iteration needs one
// multi-column band solve, one B product, two Gram matrices and a small dense eigenproblem
// (parallel cyclic Jacobi in LDS).  Eigen-residuals and the threshold test are FP64.
#include <atomic>
#include <thread>
#include <cmath>

#include "gx_internal.h"

namespace gx {

constexpr int MAXM = 48;                       // eigensolver block size limit (multiple of 8)
constexpr int MSTART = 32;                     // threshold mode: first block (one solve panel)

__device__ inline bool has_bit(const uint64_t* mask, int64_t item, int W, int j) {
  return (mask[item * W + j / 64] >> (j % 64)) & 1ull;
}
__device__ inline int popc_mask(const uint64_t* mask, int64_t item, int W) {
  int c = 0;
  for (int w = 0; w < W; ++w) c += __popcll(mask[item * W + w]);
  return c;
}
// partition-of-unity weight of node n in subdomain j (zero off the interior)
__device__ inline double pou(const int32_t* I_loc, const int32_t* cnt, int64_t N, int j,
                             int64_t n) {
  return I_loc[(int64_t)j * N + n] >= 0 ? 1.0 / cnt[n] : 0.0;
}

struct GeneoDev {
  const int32_t* conn;
  const int32_t* ne_ptr;
  const int32_t* ne_idx;
  const double* Ke;
  const uint8_t* fixed;
  const uint64_t* emask;
  int W;
  int64_t N;
  const int32_t* D_nodes;
  const int64_t* offD;
  const int64_t* nD;
  const int32_t* D_loc;
  const int32_t* I_loc;
  const int32_t* cnt;
};

// diagonal of M_j = A^N + sigma X A^o X on the Neumann DOFs (1 on clamped DOFs)
__global__ void k_neumann_diag(GeneoDev g, double sigma, const int64_t* doff, double* dM) {
  const int j = blockIdx.y;
  const int64_t ln = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ln >= g.nD[j]) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  const double xn = pou(g.I_loc, g.cnt, g.N, j, n);
  double d0 = 0, d1 = 0, d2 = 0;
  for (int k = g.ne_ptr[n]; k < g.ne_ptr[n + 1]; ++k) {
    const int64_t e = g.ne_idx[k];
    if (!has_bit(g.emask, e, g.W, j)) continue;
    const double w = popc_mask(g.emask, e, g.W) >= 2 ? 1.0 + sigma * xn * xn : 1.0;
    int a = 0;
    while (a < 19 && g.conn[20 * e + a] != n) ++a;
    const double* kb = g.Ke + ((e * 20 + a) * 20 + a) * 9;
    d0 += w * kb[0];
    d1 += w * kb[4];
    d2 += w * kb[8];
  }
  double* o = dM + doff[j] + 3 * ln;
  o[0] = g.fixed[3 * n] ? 1.0 : d0;
  o[1] = g.fixed[3 * n + 1] ? 1.0 : d1;
  o[2] = g.fixed[3 * n + 2] ? 1.0 : d2;
}

// M_j = A^N + sigma X A^o X in band storage over the Neumann DOFs; clamped DOFs -> identity.
// The band is zero-filled first; one 64-thread work-group per (node, subdomain) then sums
// the node's three rows over its elements in the subdomain (element order, deterministic)
// into the node's block row of K's pattern in LDS, and writes the blocks whose column node
// is in the subdomain and lies on or below the diagonal, scaled symmetrically by
// diag(M)^-1/2 when dM is given (FP32 factors).  Only the nonzero blocks are written.
constexpr int NROW = 128;                        // blocks in one block row of K, at most

template <class T>
__global__ void __launch_bounds__(64) k_neumann_fill(GeneoDev g, const int32_t* rp,
                                                     const int32_t* colk, double sigma,
                                                     BandView bv, const int64_t* doff,
                                                     const double* dM, T* v, int* err) {
  __shared__ double rv[NROW * 9];
  __shared__ int32_t rc[NROW];
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j]) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  const int64_t B = bv.B[j], ld = bv.ld[j];
  T* base = v + bv.off[j];
  const int rb = rp[n], len = rp[n + 1] - rb;
  if (len > NROW) {
    if (threadIdx.x == 0) atomicOr(err, 1);
    return;
  }
  for (int i = threadIdx.x; i < len; i += 64) rc[i] = colk[rb + i];
  for (int i = threadIdx.x; i < len * 9; i += 64) rv[i] = 0.0;
  __syncthreads();
  const double xn = pou(g.I_loc, g.cnt, g.N, j, n);
  for (int k = g.ne_ptr[n]; k < g.ne_ptr[n + 1]; ++k) {
    const int64_t e = g.ne_idx[k];
    if (!has_bit(g.emask, e, g.W, j)) continue;
    const bool over = popc_mask(g.emask, e, g.W) >= 2;
    int a = 0;
    while (a < 19 && g.conn[20 * e + a] != n) ++a;
    for (int t = threadIdx.x; t < 180; t += 64) {
      const int b = t / 9, comp = t - 9 * (t / 9);
      const int m = g.conn[20 * e + b];
      int lo = 0, hi = len - 1;                    // m's block in the row (sorted columns)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rc[mid] < m) lo = mid + 1; else hi = mid;
      }
      const double w = over ? 1.0 + sigma * xn * pou(g.I_loc, g.cnt, g.N, j, m) : 1.0;
      rv[9 * lo + comp] += w * g.Ke[((e * 20 + a) * 20 + b) * 9 + comp];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < len * 9; idx += 64) {
    const int sl = idx / 9, comp = idx - 9 * (idx / 9);
    const int i = comp / 3, kk = comp - 3 * (comp / 3);
    const int64_t m = rc[sl];
    const int64_t lm = g.D_loc[(int64_t)j * g.N + m];
    if (lm < 0) continue;
    const int64_t row = 3 * ln + i, col = 3 * lm + kk;
    const int64_t o = col - row + B;
    if (col > row || o < 0) continue;
    double val = rv[idx];
    if (g.fixed[3 * n + i] || g.fixed[3 * m + kk]) val = (row == col) ? 1.0 : 0.0;
    if (dM) val /= sqrt(dM[doff[j] + row] * dM[doff[j] + col]);
    base[row * ld + o] = (T)val;
  }
}

// T = MX - theta BX (per-column Ritz values), active subdomains only
__global__ void k_res_block(const int64_t* nrows, int m, const int64_t* voff,
                            const int32_t* active, const double* theta, const double* MX,
                            const double* BX, double* T) {
  const int j = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!active[j] || r >= 3 * nrows[j] * m) return;
  const int64_t i = voff[j] + r;
  T[i] = MX[i] - theta[(int64_t)j * MAXM + r % m] * BX[i];
}

// Y = X - T, active subdomains only
__global__ void k_sub_block(const int64_t* nrows, int m, const int64_t* voff,
                            const int32_t* active, const double* X, const double* T,
                            double* Y) {
  const int j = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!active[j] || r >= 3 * nrows[j] * m) return;
  Y[voff[j] + r] = X[voff[j] + r] - T[voff[j] + r];
}

// dst = src * diag^-1/2 (row scaling of the m columns), active subdomains only
__global__ void k_scale_rows(const int64_t* nrows, int m, const int64_t* voff,
                             const int64_t* doff, const int32_t* active, const double* dM,
                             const double* src, double* dst) {
  const int j = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!active[j] || r >= 3 * nrows[j] * m) return;
  dst[voff[j] + r] = src[voff[j] + r] / sqrt(dM[doff[j] + r / m]);
}

// Y = X_j A^o X_j X for the m columns of subdomain j (row-major, lane = column)
// B = X A^o X on the Neumann DOFs of each subdomain, stored once as node block rows over
// K's pattern (the blocks of row (j, node) at brow[offD[j] + ln], 9 values each, zero where
// no overlap element of j connects the two nodes or a DOF is clamped), so that each B
// product reads every block once instead of re-reading element matrices and solution rows
// per element
__global__ void k_brow_len(GeneoDev g, const int32_t* rp, int64_t* len) {
  const int j = blockIdx.y;
  const int64_t ln = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ln >= g.nD[j]) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  len[g.offD[j] + ln] = rp[n + 1] - rp[n];
}

__global__ void __launch_bounds__(64) k_b_fill(GeneoDev g, const int32_t* rp,
                                               const int32_t* colk, const int64_t* brow,
                                               double* bv) {
  __shared__ double rv[NROW * 9];
  __shared__ int32_t rc[NROW];
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j]) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  const int rb = rp[n], len = rp[n + 1] - rb;      // <= NROW (checked by the Neumann fill)
  for (int i = threadIdx.x; i < len; i += 64) rc[i] = colk[rb + i];
  for (int i = threadIdx.x; i < len * 9; i += 64) rv[i] = 0.0;
  __syncthreads();
  const double xn = pou(g.I_loc, g.cnt, g.N, j, n);
  if (xn != 0.0)
    for (int k = g.ne_ptr[n]; k < g.ne_ptr[n + 1]; ++k) {
      const int64_t e = g.ne_idx[k];
      if (!has_bit(g.emask, e, g.W, j) || popc_mask(g.emask, e, g.W) < 2) continue;
      int a = 0;
      while (a < 19 && g.conn[20 * e + a] != n) ++a;
      for (int t = threadIdx.x; t < 180; t += 64) {
        const int b = t / 9, comp = t - 9 * (t / 9);
        const int m = g.conn[20 * e + b];
        int lo = 0, hi = len - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (rc[mid] < m) lo = mid + 1; else hi = mid;
        }
        rv[9 * lo + comp] += xn * pou(g.I_loc, g.cnt, g.N, j, m) *
                             g.Ke[((e * 20 + a) * 20 + b) * 9 + comp];
      }
      __syncthreads();
    }
  double* out = bv + 9 * brow[g.offD[j] + ln];
  for (int idx = threadIdx.x; idx < len * 9; idx += 64) {
    const int sl = idx / 9, comp = idx - 9 * (idx / 9);
    const int64_t m = rc[sl];
    const bool fx = g.fixed[3 * n + comp / 3] || g.fixed[3 * m + comp % 3];
    out[idx] = fx ? 0.0 : rv[idx];
  }
}

// A^N of each subdomain as node block rows over K's pattern, laid out like B: the sum of
// the element matrices of the subdomain's elements, with the rows and columns of clamped
// DOFs zero (the product puts X back on clamped rows).  Used by the mixed path, which
// forms M X explicitly.
__global__ void __launch_bounds__(64) k_a_fill(GeneoDev g, const int32_t* rp,
                                               const int32_t* colk, const int64_t* brow,
                                               double* av) {
  __shared__ double rv[NROW * 9];
  __shared__ int32_t rc[NROW];
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j]) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  const int rb = rp[n], len = rp[n + 1] - rb;      // <= NROW (checked by the Neumann fill)
  for (int i = threadIdx.x; i < len; i += 64) rc[i] = colk[rb + i];
  for (int i = threadIdx.x; i < len * 9; i += 64) rv[i] = 0.0;
  __syncthreads();
  for (int k = g.ne_ptr[n]; k < g.ne_ptr[n + 1]; ++k) {
    const int64_t e = g.ne_idx[k];
    if (!has_bit(g.emask, e, g.W, j)) continue;
    int a = 0;
    while (a < 19 && g.conn[20 * e + a] != n) ++a;
    for (int t = threadIdx.x; t < 180; t += 64) {  // distinct nodes b: distinct slots
      const int b = t / 9, comp = t - 9 * (t / 9);
      const int mnode = g.conn[20 * e + b];
      int lo = 0, hi = len - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rc[mid] < mnode) lo = mid + 1; else hi = mid;
      }
      rv[9 * lo + comp] += g.Ke[((e * 20 + a) * 20 + b) * 9 + comp];
    }
    __syncthreads();
  }
  double* out = av + 9 * brow[g.offD[j] + ln];
  for (int idx = threadIdx.x; idx < len * 9; idx += 64) {
    const int sl = idx / 9, comp = idx - 9 * (idx / 9);
    const int64_t mnode = rc[sl];
    const bool fx = g.fixed[3 * n + comp / 3] || g.fixed[3 * mnode + comp % 3];
    out[idx] = fx ? 0.0 : rv[idx];
  }
}

// The blocks of each stored row of B that can contribute: nonzero, with a column node
// among the subdomain's Neumann nodes.  One 64-lane work-group per row, lanes over the
// row's slots (at most NROW = 128); k_bcount writes each row's count, k_bcompact (after an
// exclusive scan of the counts) copies those blocks in slot order with the column node's
// local index.
__device__ inline bool b_keep(const GeneoDev& g, const int32_t* colk, const double* bv,
                              int j, int rb, int64_t b0, int sl, int len, int32_t* lm_out) {
  if (sl >= len) return false;
  const int32_t lm = g.D_loc[(int64_t)j * g.N + colk[rb + sl]];
  *lm_out = lm;
  if (lm < 0) return false;
  const double* kb = bv + 9 * (b0 + sl);
  bool nz = false;
#pragma unroll
  for (int c = 0; c < 9; ++c) nz = nz || kb[c] != 0.0;
  return nz;
}

__global__ void __launch_bounds__(64) k_bcount(GeneoDev g, const int32_t* rp,
                                               const int32_t* colk, const int64_t* brow,
                                               const double* bv, int64_t* cnt) {
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j]) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  const int rb = rp[n], len = rp[n + 1] - rb;
  const int64_t b0 = brow[g.offD[j] + ln];
  int c = 0;
  for (int base = 0; base < len; base += 64) {
    int32_t lm = -1;
    c += __popcll(__ballot(b_keep(g, colk, bv, j, rb, b0, base + (int)threadIdx.x, len, &lm)));
  }
  if (threadIdx.x == 0) cnt[g.offD[j] + ln] = c;
}

__global__ void __launch_bounds__(64) k_bcompact(GeneoDev g, const int32_t* rp,
                                                 const int32_t* colk, const int64_t* brow,
                                                 const double* bv, const int64_t* crow,
                                                 int32_t* cloc, double* cbv) {
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j]) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  const int rb = rp[n], len = rp[n + 1] - rb;
  const int64_t b0 = brow[g.offD[j] + ln];
  int64_t o = crow[g.offD[j] + ln];
  const int lane = threadIdx.x;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;   // lanes < this one
  for (int base = 0; base < len; base += 64) {
    int32_t lm = -1;
    const bool keep = b_keep(g, colk, bv, j, rb, b0, base + lane, len, &lm);
    const uint64_t mask = __ballot(keep);
    if (keep) {
      const int64_t d = o + __popcll(mask & below);
      cloc[d] = lm;
#pragma unroll
      for (int c = 0; c < 9; ++c) cbv[9 * d + c] = bv[9 * (b0 + base + lane) + c];
    }
    o += __popcll(mask);
  }
}

// (y0, y1, y2) = row ln of S X for a compact block-row operator S (lane = column): each
// lane holds two of the row's local column indices, handed to all lanes by a lane read,
// and the X rows of 8 blocks are loaded before any is used.  Blocks are summed in slot
// order.
__device__ inline void rows_product(const int64_t* crow, const int32_t* cloc, const double* cbv,
                                    int64_t r, int m, const double* Xj, int lane, double& y0,
                                    double& y1, double& y2) {
  const int64_t c0 = crow[r];
  const int cnt = (int)(crow[r + 1] - c0);         // <= NROW
  const int32_t la = lane < cnt ? cloc[c0 + lane] : 0;
  const int32_t lb = lane + 64 < cnt ? cloc[c0 + 64 + lane] : 0;
  const double* kb0 = cbv + 9 * c0;
  const int col = min(lane, m - 1);                // lanes past m repeat a column, unstored
  y0 = y1 = y2 = 0.0;
  for (int s0 = 0; s0 < cnt; s0 += 8) {
    double xv[8][3];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sl = min(s0 + q, cnt - 1);
      const int64_t lm = sl < 64 ? __shfl(la, sl) : __shfl(lb, sl - 64);
#pragma unroll
      for (int c = 0; c < 3; ++c) xv[q][c] = Xj[(3 * lm + c) * m + col];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (s0 + q >= cnt) break;
      const double* kb = kb0 + 9 * (s0 + q);
      y0 += kb[0] * xv[q][0] + kb[1] * xv[q][1] + kb[2] * xv[q][2];
      y1 += kb[3] * xv[q][0] + kb[4] * xv[q][1] + kb[5] * xv[q][2];
      y2 += kb[6] * xv[q][0] + kb[7] * xv[q][1] + kb[8] * xv[q][2];
    }
  }
}

// Y = B X for the m columns of the active subdomains, from the compact rows of B
__global__ void __launch_bounds__(64) k_bmul_rows(GeneoDev g, const int64_t* crow,
                                                  const int32_t* cloc, const double* cbv,
                                                  int m, const int64_t* voff,
                                                  const int32_t* active, const double* X,
                                                  double* Y) {
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j] || !active[j]) return;
  const int lane = threadIdx.x;
  double y0, y1, y2;
  rows_product(crow, cloc, cbv, g.offD[j] + ln, m, X + voff[j], lane, y0, y1, y2);
  if (lane < m) {
    double* Yj = Y + voff[j];
    Yj[(3 * ln) * m + lane] = y0;
    Yj[(3 * ln + 1) * m + lane] = y1;
    Yj[(3 * ln + 2) * m + lane] = y2;
  }
}

// Y = A^N X + sigma BX for the m columns of the active subdomains, from the compact rows of
// A^N; clamped rows take X (the pencil carries identity rows there)
__global__ void __launch_bounds__(64) k_amul_rows(GeneoDev g, const int64_t* crow,
                                                  const int32_t* cloc, const double* cbv,
                                                  int m, const int64_t* voff,
                                                  const int32_t* active, const double* X,
                                                  const double* BX, double sigma, double* Y) {
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j] || !active[j]) return;
  const int lane = threadIdx.x;
  const double* Xj = X + voff[j];
  double y[3];
  rows_product(crow, cloc, cbv, g.offD[j] + ln, m, Xj, lane, y[0], y[1], y[2]);
  if (lane < m) {
    const int64_t n = g.D_nodes[g.offD[j] + ln];
    const double* BXj = BX + voff[j];
    double* Yj = Y + voff[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int64_t e = (3 * ln + c) * m + lane;
      Yj[e] = g.fixed[3 * n + c] ? Xj[e] : y[c] + sigma * BXj[e];
    }
  }
}

// deterministic pseudo-random start block (splitmix64 of the entry index), zero on clamps
__global__ void k_rand_init(GeneoDev g, int m, const int64_t* voff, double* X) {
  const int j = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 3 * g.nD[j] * m) return;
  const int64_t row = r / m;
  const int64_t n = g.D_nodes[g.offD[j] + row / 3];
  uint64_t z = (uint64_t)r + 0x9E3779B97F4A7C15ull * (uint64_t)(j + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
  X[voff[j] + r] = g.fixed[3 * n + row % 3] ? 0.0 : u;
}

// the m0 columns of a block into the first m0 columns of a block of m1 >= m0 columns
__global__ void k_widen(const int64_t* nrows, int m0, const int64_t* voff0, const double* X0,
                        int m1, const int64_t* voff1, double* X1) {
  const int j = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nrows[j] * m0) return;
  const int64_t row = e / m0, c = e - row * m0;
  X1[voff1[j] + row * m1 + c] = X0[voff0[j] + e];
}

__global__ void k_copy_active(int64_t n_rows_max, const int64_t* nrows, int m,
                              const int64_t* voff, const int32_t* active, const double* src,
                              double* dst) {
  const int j = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!active[j] || r >= 3 * nrows[j] * m) return;
  dst[voff[j] + r] = src[voff[j] + r];
}

// Gram partials G_U[a][b] = sum_i U[i][a] V1[i][b] and G_2 = sum_i U[i][a] V2[i][b] over a
// chunk of rows; chunk partials are reduced in a fixed order afterwards
constexpr int GCH = 4096;
constexpr int GROWS = 32;
__global__ void __launch_bounds__(256) k_gram(const int64_t* nrows, int m, const int64_t* voff,
                                              const int32_t* active, const double* U,
                                              const double* V1, const double* V2,
                                              int64_t nch_max, double* part) {
  __shared__ double su[GROWS][MAXM], s1[GROWS][MAXM], s2[GROWS][MAXM];
  const int j = blockIdx.y;
  if (!active[j]) return;
  const int64_t n3 = 3 * nrows[j];
  const int64_t r0 = (int64_t)blockIdx.x * GCH;
  constexpr int EPT = (MAXM * MAXM + 255) / 256;
  double a1[EPT], a2[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) a1[q] = a2[q] = 0.0;
  const double* Uj = U + voff[j];
  const double* V1j = V1 + voff[j];
  const double* V2j = V2 + voff[j];
  for (int64_t rb = r0; rb < min(n3, r0 + GCH); rb += GROWS) {
    for (int t = threadIdx.x; t < GROWS * m; t += 256) {
      const int rr = t / m, cc = t % m;
      const int64_t row = rb + rr;
      const bool ok = row < n3;
      su[rr][cc] = ok ? Uj[row * m + cc] : 0.0;
      s1[rr][cc] = ok ? V1j[row * m + cc] : 0.0;
      s2[rr][cc] = ok ? V2j[row * m + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < m * m) {
        const int a = e / m, b = e % m;
        double t1 = 0, t2 = 0;
        for (int rr = 0; rr < GROWS; ++rr) {
          t1 += su[rr][a] * s1[rr][b];
          t2 += su[rr][a] * s2[rr][b];
        }
        a1[q] += t1;
        a2[q] += t2;
      }
    }
    __syncthreads();
  }
  double* pj = part + ((int64_t)j * nch_max + blockIdx.x) * 2 * MAXM * MAXM;
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + 256 * q;
    if (e < m * m) {
      pj[e] = a1[q];
      pj[MAXM * MAXM + e] = a2[q];
    }
  }
}

__global__ void k_gram_sum(const int64_t* nrows, int m, const int32_t* active,
                           int64_t nch_max, const double* part, double* G) {
  const int j = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (!active[j] || e >= 2 * MAXM * MAXM) return;
  const int64_t nch = (3 * nrows[j] + GCH - 1) / GCH;
  double s = 0.0;
  for (int64_t k = 0; k < nch; ++k) s += part[((int64_t)j * nch_max + k) * 2 * MAXM * MAXM + e];
  G[(int64_t)j * 2 * MAXM * MAXM + e] = s;
}

// Small dense Rayleigh-Ritz per subdomain: G_B c = mu G_M c, largest mu first.
// G layout: [G_M (m x m, ld m) | G_B] inside a 2 MAXM^2 slot.  Output: c (m x m row-major,
// column b = b-th Ritz vector) and theta_b = 1 / mu_b.
__global__ void __launch_bounds__(256) k_rayleigh_ritz(int m, const int32_t* active,
                                                       const double* G, double* Cout,
                                                       double* theta, int* err) {
  __shared__ double L[MAXM][MAXM + 1], H[MAXM][MAXM + 1], T[MAXM][MAXM + 1],
      V[MAXM][MAXM + 1];
  __shared__ double dsc[MAXM], rc[MAXM / 2 + 1], rs[MAXM / 2 + 1], mu[MAXM];
  __shared__ int rp[MAXM / 2 + 1], rq[MAXM / 2 + 1], perm[MAXM];
  __shared__ double offn;
  const int j = blockIdx.x;
  if (!active[j]) return;
  const int t = threadIdx.x;
  const double* Gj = G + (int64_t)j * 2 * MAXM * MAXM;
  for (int e = t; e < m * m; e += 256) {
    const int a = e / m, b = e % m;
    L[a][b] = 0.5 * (Gj[a * m + b] + Gj[b * m + a]);
    T[a][b] = 0.5 * (Gj[MAXM * MAXM + a * m + b] + Gj[MAXM * MAXM + b * m + a]);
  }
  __syncthreads();
  if (t < m) dsc[t] = L[t][t] > 0 ? 1.0 / sqrt(L[t][t]) : 0.0;
  __syncthreads();
  for (int e = t; e < m * m; e += 256) {
    const int a = e / m, b = e % m;
    L[a][b] *= dsc[a] * dsc[b];
    T[a][b] *= dsc[a] * dsc[b];
  }
  __syncthreads();
  // Cholesky of the scaled M-Gram (lower, in place)
  for (int i = 0; i < m; ++i) {
    if (t == 0) {
      double d = L[i][i];
      if (!(d > 1e-13)) {
        atomicOr(err, 1);
        d = 1.0;
      }
      L[i][i] = sqrt(d);
    }
    __syncthreads();
    for (int r = i + 1 + t; r < m; r += 256) L[r][i] /= L[i][i];
    __syncthreads();
    const int mm = m - i - 1;
    for (int e = t; e < mm * mm; e += 256) {
      const int r = i + 1 + e / mm, s = i + 1 + e % mm;
      if (s <= r) L[r][s] -= L[r][i] * L[s][i];
    }
    __syncthreads();
  }
  // H = L^-1 G_B L^-T: first W = L^-1 G_B (column k by thread k), then H = L^-1 W^T
  if (t < m) {
    for (int i = 0; i < m; ++i) {
      double s = T[i][t];
      for (int l = 0; l < i; ++l) s -= L[i][l] * H[l][t];
      H[i][t] = s / L[i][i];
    }
  }
  __syncthreads();
  if (t < m) {
    for (int i = 0; i < m; ++i) {
      double s = H[t][i];
      for (int l = 0; l < i; ++l) s -= L[i][l] * T[l][t];
      T[i][t] = s / L[i][i];
    }
  }
  __syncthreads();
  for (int e = t; e < m * m; e += 256) {
    const int a = e / m, b = e % m;
    H[a][b] = 0.5 * (T[a][b] + T[b][a]);
    V[a][b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  // parallel cyclic Jacobi, round-robin pairing (one index is a dummy when m is odd)
  const int me = m + (m & 1);
  const int np = me / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (t == 0) {
      double off = 0.0, all = 0.0;
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
          all += H[a][b] * H[a][b];
          if (a != b) off += H[a][b] * H[a][b];
        }
      offn = (off <= 1e-30 * all) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (offn != 0.0) break;
    for (int round = 0; round < me - 1; ++round) {
      if (t < np) {
        int p, q;
        if (t == 0) {
          p = me - 1;
          q = round;
        } else {
          p = (round + t) % (me - 1);
          q = (round - t + (me - 1)) % (me - 1);
        }
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        double c = 1.0, s = 0.0;
        if (q < m && H[p][q] != 0.0) {
          const double th = (H[q][q] - H[p][p]) / (2.0 * H[p][q]);
          const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(tt * tt + 1.0);
          s = tt * c;
        }
        rp[t] = p;
        rq[t] = q < m ? q : p;
        rc[t] = c;
        rs[t] = s;
      }
      __syncthreads();
      for (int e = t; e < np * m; e += 256) {      // rows: H <- P^T H
        const int k = e / m, col = e % m;
        const int p = rp[k], q = rq[k];
        if (p == q) continue;
        const double c = rc[k], s = rs[k];
        const double hp = H[p][col], hq = H[q][col];
        H[p][col] = c * hp - s * hq;
        H[q][col] = s * hp + c * hq;
      }
      __syncthreads();
      for (int e = t; e < np * m; e += 256) {      // columns: H <- H P, V <- V P
        const int k = e / m, row = e % m;
        const int p = rp[k], q = rq[k];
        if (p == q) continue;
        const double c = rc[k], s = rs[k];
        const double hp = H[row][p], hq = H[row][q];
        H[row][p] = c * hp - s * hq;
        H[row][q] = s * hp + c * hq;
        const double vp = V[row][p], vq = V[row][q];
        V[row][p] = c * vp - s * vq;
        V[row][q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  // order by decreasing mu
  if (t == 0) {
    for (int a = 0; a < m; ++a) {
      mu[a] = H[a][a];
      perm[a] = a;
    }
    for (int a = 0; a < m; ++a)
      for (int b = a + 1; b < m; ++b)
        if (mu[perm[b]] > mu[perm[a]]) {
          const int tmp = perm[a];
          perm[a] = perm[b];
          perm[b] = tmp;
        }
  }
  __syncthreads();
  // c = D L^-T V (column b = Ritz vector of the b-th largest mu)
  if (t < m) {
    const int src = perm[t];
    for (int i = m - 1; i >= 0; --i) {
      double s = V[i][src];
      for (int l = i + 1; l < m; ++l) s -= L[l][i] * T[l][t];
      T[i][t] = s / L[i][i];
    }
    theta[(int64_t)j * MAXM + t] = 1.0 / mu[src];
  }
  __syncthreads();
  for (int e = t; e < m * m; e += 256) {
    const int a = e / m, b = e % m;
    Cout[(int64_t)j * MAXM * MAXM + a * m + b] = dsc[a] * T[a][b];
  }
}

// out[i][b] = sum_a in[i][a] c[a][b] (row-major blocks of m columns).  A work-group takes
// ROT_ROWS rows, so that the m x m matrix it stages in LDS serves many of them; each wave
// forms four rows at a time (lane = column).
constexpr int ROT_ROWS = 64;
__global__ void __launch_bounds__(256) k_rotate(const int64_t* nrows, int m,
                                                const int64_t* voff, const int32_t* active,
                                                const double* Cm, const double* in,
                                                double* out) {
  __shared__ double c[MAXM][MAXM];
  const int j = blockIdx.y;
  if (!active[j]) return;
  const int64_t n3 = 3 * nrows[j];
  const int64_t r0 = (int64_t)blockIdx.x * ROT_ROWS;
  if (r0 >= n3) return;
  for (int e = threadIdx.x; e < m * m; e += 256) c[e / m][e % m] = Cm[(int64_t)j * MAXM * MAXM + e];
  __syncthreads();
  const int b = threadIdx.x % 64, w = threadIdx.x / 64;
  const int bb = min(b, m - 1);
  const int64_t rend = min(n3, r0 + ROT_ROWS);
  const double* base = in + voff[j];
  for (int64_t row = r0 + w; row < rend; row += 16) {   // rows row + 4 q, q < 4
    // lane a loads entry a of each row (one coalesced load per row); the products take
    // entry a from lane a (a wave-uniform lane read into a scalar operand)
    double xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) xv[q] = base[min(row + 4 * q, rend - 1) * m + bb];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < m; ++a) {
      const double ca = c[a][bb];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += lane_value(xv[q], a) * ca;
    }
    if (b < m)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (row + 4 * q < rend) out[voff[j] + (row + 4 * q) * m + b] = acc[q];
  }
}

// per column: ||MX - theta BX||^2, ||MX||^2 and ||X||^2 (chunk partials, then fixed-order
// sums)
__global__ void __launch_bounds__(256) k_resid(const int64_t* nrows, int m,
                                               const int64_t* voff, const int32_t* active,
                                               const double* theta, const double* MX,
                                               const double* BX, const double* X,
                                               int64_t nch_max, double* part) {
  __shared__ double red[4][3][64];
  const int j = blockIdx.y;
  if (!active[j]) return;
  const int64_t n3 = 3 * nrows[j];
  const int b = threadIdx.x % 64, rg = threadIdx.x / 64;
  double r2 = 0, m2 = 0, x2 = 0;
  if (b < m) {
    const double th = theta[(int64_t)j * MAXM + b];
    const int64_t r0 = (int64_t)blockIdx.x * GCH;
    for (int64_t row = r0 + rg; row < min(n3, r0 + GCH); row += 4) {
      const int64_t e = voff[j] + row * m + b;
      const double mx = MX[e];
      const double d = mx - th * BX[e];
      r2 += d * d;
      m2 += mx * mx;
      x2 += X[e] * X[e];
    }
  }
  red[rg][0][b] = r2;
  red[rg][1][b] = m2;
  red[rg][2][b] = x2;
  __syncthreads();
  if (rg == 0 && b < m) {
    double* pj = part + ((int64_t)j * nch_max + blockIdx.x) * 3 * MAXM;
#pragma unroll
    for (int q = 0; q < 3; ++q)
      pj[q * MAXM + b] = red[0][q][b] + red[1][q][b] + red[2][q][b] + red[3][q][b];
  }
}

__global__ void k_resid_sum(const int64_t* nrows, const int32_t* active, int64_t nch_max,
                            const double* part, double* out) {
  const int j = blockIdx.x;
  const int e = threadIdx.x;
  if (!active[j] || e >= 3 * MAXM) return;
  const int64_t nch = (3 * nrows[j] + GCH - 1) / GCH;
  double s = 0.0;
  for (int64_t k = 0; k < nch; ++k) s += part[((int64_t)j * nch_max + k) * 3 * MAXM + e];
  out[(int64_t)j * 3 * MAXM + e] = s;
}

// ---------------------------------------------------------------------------------------
// coarse space
struct CoarseDev {
  const int32_t* I_nodes;
  const int64_t* offI;
  const int64_t* nI;
  const int64_t* zoff;        // Z_j column-major, 3 nI_j rows
  const int32_t* nev;
  const int32_t* coff;
};

__global__ void k_build_Z(GeneoDev g, CoarseDev cd, int m, const int64_t* voff,
                          const double* X, double* Z) {
  const int j = blockIdx.y;
  const int64_t li = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n3 = 3 * cd.nI[j];
  if (li >= n3) return;
  const int64_t n = cd.I_nodes[cd.offI[j] + li / 3];
  const int64_t ld = 3 * (int64_t)g.D_loc[(int64_t)j * g.N + n] + li % 3;
  const double w = g.fixed[3 * n + li % 3] ? 0.0 : 1.0 / g.cnt[n];
  for (int a = 0; a < cd.nev[j]; ++a)
    Z[cd.zoff[j] + (int64_t)a * n3 + li] = w * X[voff[j] + ld * m + a];
}

// V_j = K R_j^T Z_j on the Neumann rows of j (row-major, nev_j columns, lane = column)
__global__ void __launch_bounds__(64) k_coarse_V(GeneoDev g, CoarseDev cd, const int32_t* rp,
                                                 const int32_t* col, const double* val,
                                                 const double* Z, const int64_t* vcoff,
                                                 double* Vc) {
  const int j = blockIdx.y;
  const int64_t ln = blockIdx.x;
  if (ln >= g.nD[j]) return;
  const int a = threadIdx.x, m = cd.nev[j];
  if (a >= m) return;
  const int64_t n = g.D_nodes[g.offD[j] + ln];
  const int64_t n3 = 3 * cd.nI[j];
  const double* Zj = Z + cd.zoff[j] + (int64_t)a * n3;
  double y0 = 0, y1 = 0, y2 = 0;
  for (int k = rp[n]; k < rp[n + 1]; ++k) {
    const int64_t mm = col[k];
    const int64_t li = g.I_loc[(int64_t)j * g.N + mm];
    if (li < 0) continue;
    const double* kb = val + (int64_t)k * 9;
    const double z0 = Zj[3 * li], z1 = Zj[3 * li + 1], z2 = Zj[3 * li + 2];
    y0 += kb[0] * z0 + kb[1] * z1 + kb[2] * z2;
    y1 += kb[3] * z0 + kb[4] * z1 + kb[5] * z2;
    y2 += kb[6] * z0 + kb[7] * z1 + kb[8] * z2;
  }
  double* o = Vc + vcoff[j];
  o[(3 * ln) * m + a] = y0;
  o[(3 * ln + 1) * m + a] = y1;
  o[(3 * ln + 2) * m + a] = y2;
}

__global__ void k_pair_adjacency(const uint64_t* nand, const uint64_t* nor, int W, int64_t N,
                                 int n_sub, int32_t* adj) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  for (int wk = 0; wk < W; ++wk) {
    uint64_t bk = nand[n * W + wk];
    while (bk) {
      const int k = wk * 64 + __ffsll((unsigned long long)bk) - 1;
      bk &= bk - 1;
      for (int wj = 0; wj < W; ++wj) {
        uint64_t bj = nor[n * W + wj];
        while (bj) {
          const int jj = wj * 64 + __ffsll((unsigned long long)bj) - 1;
          bj &= bj - 1;
          adj[(int64_t)k * n_sub + jj] = 1;
        }
      }
    }
  }
}

// K_0 block (k, j) = sum over nodes in I_k and D_j of Z_k^T V_j
__global__ void __launch_bounds__(256) k_coarse_pair(GeneoDev g, CoarseDev cd, int n_sub,
                                                     const int32_t* adj, const double* Z,
                                                     const double* Vc, const int64_t* vcoff,
                                                     int64_t n0, double* K0) {
  const int k = blockIdx.x, j = blockIdx.y;
  if (!adj[(int64_t)k * n_sub + j]) return;
  const int mk = cd.nev[k], mj = cd.nev[j];
  if (mk == 0 || mj == 0) return;
  constexpr int EPT = (MAXM * MAXM + 255) / 256;
  double acc[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) acc[q] = 0.0;
  const int64_t nIk = cd.nI[k], n3k = 3 * nIk;
  const double* Zk = Z + cd.zoff[k];
  const double* Vj = Vc + vcoff[j];
  for (int64_t ln = 0; ln < nIk; ++ln) {
    const int64_t n = cd.I_nodes[cd.offI[k] + ln];
    const int64_t ldj = g.D_loc[(int64_t)j * g.N + n];
    if (ldj < 0) continue;
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < mk * mj) {
        const int b = e / mj, a = e % mj;
        double s = 0.0;
        for (int c = 0; c < 3; ++c)
          s += Zk[(int64_t)b * n3k + 3 * ln + c] * Vj[(3 * ldj + c) * mj + a];
        acc[q] += s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + 256 * q;
    if (e < mk * mj) {
      const int b = e / mj, a = e % mj;
      K0[(int64_t)(cd.coff[k] + b) * n0 + cd.coff[j] + a] = acc[q];
    }
  }
}

// symmetrise K_0 into full band storage (B = n0 - 1, ld = n0)
__global__ void k_coarse_fill(int64_t n0, const double* K0, int64_t B, int64_t ld,
                              double* band) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n0 * n0) return;
  const int64_t r = e / n0, c = e % n0;
  if (c > r) return;
  band[r * ld + (c - r + B)] = 0.5 * (K0[r * n0 + c] + K0[c * n0 + r]);
}

void geneo_coarse(gx_ctx* c, const gx_geneo_opts* o, const std::function<void()>& after_factor) {
  Schwarz& sw = c->sw;
  hipStream_t s = c->stream;
  const int n_sub = sw.n_sub;
  const int64_t N = c->n_nodes;
  const double tau = o->tau > 0 ? o->tau : 0.1;
  // at most MAXM - 8 modes per subdomain fit the eigensolver block (eight guard vectors)
  const int nev_max = std::min(o->nev_max > 0 ? o->nev_max : 32, MAXM - 8);
  std::vector<int> want(n_sub, o->nev > 0 ? o->nev : 0);
  if (o->nev_per_sub)
    for (int j = 0; j < n_sub; ++j) want[j] = o->nev_per_sub[j];
  const bool fixed_count = o->nev > 0 || o->nev_per_sub;
  int mwant = fixed_count ? 0 : nev_max;
  for (int j = 0; j < n_sub; ++j) mwant = std::max(mwant, want[j]);
  GX_REQUIRE(mwant >= 1 && mwant + 8 <= MAXM, "requested modes exceed the eigensolver block");
  // shift of the pencil: tiny in FP64; in the mixed path 0.01 tau keeps A^N + sigma B well
  // enough conditioned for FP32 factors (convergence rate (lambda + s)/(lambda_m+1 + s);
  // 0.1 tau cost the 3M-DOF flat laminate one more iteration, 14 against 13)
  const double sigma = o->precision == GX_MIXED ? 0.01 * tau
                                                : (fixed_count ? 1e-4 * tau : 1e-3 * tau);
  // backward-error target: the coarse space needs the low eigenvectors to a few digits
  // only (Ritz values are then exact to about tol^2, so the selection against tau is
  // unaffected); on the 3M-DOF flat laminate and the 3M-DOF curved wrinkled L-section the
  // coarse dimension and the PCG iteration count are the same from 1e-4 to 1e-10
  const double tol = o->eig_tol > 0 ? o->eig_tol : 1e-4;
  const int maxit = o->eig_maxit > 0 ? o->eig_maxit : 1000;
  for (int j = 0; j < n_sub; ++j)
    GX_REQUIRE(3 * sw.nD[j] >= mwant + 8, "subdomain too small for the eigensolver block");
  Timer te(s);
  GeneoDev g{c->conn.p, c->ne_ptr.p, c->ne_idx.p, c->Ke.p, c->fixed.p, sw.elem_mask.p, sw.W,
             N, sw.D_nodes.p, sw.d_offD.p, sw.d_nD.p, sw.D_loc.p, sw.I_loc.p, sw.node_cnt.p};
  int64_t maxD = 0;
  for (int j = 0; j < n_sub; ++j) maxD = std::max(maxD, sw.nD[j]);
  // Neumann pencil M = A^N + sigma B in band storage, factored
  // mixed precision: FP32 factors of diag(M)^-1/2 M diag(M)^-1/2; the Rayleigh-Ritz step,
  // residuals and threshold test stay FP64 (M Y is then formed explicitly)
  const bool fp32 = o->precision == GX_MIXED;
  BandSet Mb;
  Mb.share = c->share;
  std::vector<int64_t> doff(n_sub + 1, 0);
  for (int j = 0; j < n_sub; ++j) doff[j + 1] = doff[j] + 3 * sw.nD[j];
  DevBuf<int64_t> d_doff(n_sub + 1);
  to_dev(d_doff.p, doff.data(), n_sub + 1, s);
  DevBuf<double> dM;
  {
    std::vector<int64_t> n3(n_sub), env;
    std::vector<int32_t> first;
    std::vector<int64_t> B =
        list_bandwidth(c, sw.D_nodes.p, sw.d_offD.p, sw.d_nD.p, sw.D_loc.p, sw.nD, &env, &first);
    for (int j = 0; j < n_sub; ++j) n3[j] = 3 * sw.nD[j];
    band_layout(Mb, n3, B, fp32, s, &first);
    c->neumann_envelope = 0;
    for (int64_t e : Mb.env) c->neumann_envelope += e;
    c->neumann_flops = Mb.env_flops;
    Mb.force_groups[0] = c->tune[0];
    Mb.force_groups[1] = c->tune[1];
    c->neumann_entries = Mb.total;
    BandView bv{Mb.d_B.p, Mb.d_ld.p, Mb.d_off.p};
    DevBuf<int> ferr(1);
    zero(ferr, s);
    if (fp32) {
      dM.alloc(doff[n_sub]);
      hipLaunchKernelGGL(k_neumann_diag, dim3(nblocks(maxD, 256), n_sub), dim3(256), 0, s, g,
                         sigma, d_doff.p, dM.p);
      GX_HIP(hipMemsetAsync(Mb.v32.p, 0, Mb.total * sizeof(float), s));
      hipLaunchKernelGGL(k_neumann_fill<float>, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g,
                         c->row_ptr.p, c->col.p, sigma, bv, d_doff.p, (const double*)dM.p,
                         Mb.v32.p, ferr.p);
    } else {
      GX_HIP(hipMemsetAsync(Mb.v64.p, 0, Mb.total * sizeof(double), s));
      hipLaunchKernelGGL(k_neumann_fill<double>, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g,
                         c->row_ptr.p, c->col.p, sigma, bv, d_doff.p, (const double*)nullptr,
                         Mb.v64.p, ferr.p);
    }
    GX_HIP(hipGetLastError());
    int hferr = 0;
    to_host(&hferr, ferr.p, 1, s);
    GX_REQUIRE(!hferr, "a block row of K is longer than the Neumann assembly takes");
    try {
      band_factor(Mb, s, "the shifted Neumann matrices (GenEO eigensolver)");
    } catch (const Error& e) {
      if (!fp32 || e.code != GX_ENOTSPD) throw;
      // an FP32 factor broke down: this matrix set is refactored in FP64 (reported)
      c->fp64_fallbacks |= 2;
      band_layout(Mb, n3, B, false, s, &first);
      bv = BandView{Mb.d_B.p, Mb.d_ld.p, Mb.d_off.p};
      GX_HIP(hipMemsetAsync(Mb.v64.p, 0, Mb.total * sizeof(double), s));
      hipLaunchKernelGGL(k_neumann_fill<double>, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g,
                         c->row_ptr.p, c->col.p, sigma, bv, d_doff.p, (const double*)nullptr,
                         Mb.v64.p, ferr.p);
      GX_HIP(hipGetLastError());
      band_factor(Mb, s, "the shifted Neumann matrices (GenEO eigensolver)");
    }
  }
  if (after_factor) after_factor();
  const bool m32 = Mb.fp32;
  // B as stored node block rows (see k_b_fill)
  int64_t sumD = 0;
  for (int j = 0; j < n_sub; ++j) sumD += sw.nD[j];
  DevBuf<int64_t> brow(sumD + 1), crow(sumD + 1), crowA(m32 ? sumD + 1 : 0);
  DevBuf<double> Bv, cbv, cbvA;                    // cbvA, clocA: compact A^N rows (mixed)
  DevBuf<int32_t> cloc, clocA;
  {
    zero(brow, s);
    hipLaunchKernelGGL(k_brow_len, dim3(nblocks(maxD, 256), n_sub), dim3(256), 0, s, g,
                       c->row_ptr.p, brow.p);
    DevBuf<int64_t> stmp(scan_tmp_size(sumD + 1));
    const int64_t nbl = exclusive_scan(brow.p, sumD + 1, stmp.p, s);
    Bv.alloc(std::max<int64_t>(9 * nbl, 1));
    hipLaunchKernelGGL(k_b_fill, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g, c->row_ptr.p,
                       c->col.p, brow.p, Bv.p);
    // compact rows: the blocks that can contribute, with their local column indices
    zero(crow, s);
    hipLaunchKernelGGL(k_bcount, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g, c->row_ptr.p,
                       c->col.p, brow.p, Bv.p, crow.p);
    const int64_t nbc = exclusive_scan(crow.p, sumD + 1, stmp.p, s);
    cloc.alloc(std::max<int64_t>(nbc, 1));
    cbv.alloc(std::max<int64_t>(9 * nbc, 1));
    hipLaunchKernelGGL(k_bcompact, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g,
                       c->row_ptr.p, c->col.p, brow.p, Bv.p, crow.p, cloc.p, cbv.p);
    GX_HIP(hipGetLastError());
    if (m32) {                                     // A^N rows, the same way (mixed path)
      Bv.release();
      Bv.alloc(std::max<int64_t>(9 * nbl, 1));
      hipLaunchKernelGGL(k_a_fill, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g,
                         c->row_ptr.p, c->col.p, brow.p, Bv.p);
      zero(crowA, s);
      hipLaunchKernelGGL(k_bcount, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g,
                         c->row_ptr.p, c->col.p, brow.p, Bv.p, crowA.p);
      const int64_t nac = exclusive_scan(crowA.p, sumD + 1, stmp.p, s);
      clocA.alloc(std::max<int64_t>(nac, 1));
      cbvA.alloc(std::max<int64_t>(9 * nac, 1));
      hipLaunchKernelGGL(k_bcompact, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g,
                         c->row_ptr.p, c->col.p, brow.p, Bv.p, crowA.p, clocA.p, cbvA.p);
      GX_HIP(hipGetLastError());
    }
    GX_HIP(hipStreamSynchronize(s));
    Bv.release();
    brow.release();
  }
  // block size: a fixed count takes the wanted count + 8 guard vectors, rounded up to a
  // multiple of 8 (the multi-right-hand-side solves are built for them).  A threshold starts
  // with one full solve panel (MSTART columns: the solves cost about the same per iteration
  // at any width up to it) and grows to nev_max + 16 as soon as more than m - 8 Ritz values
  // lie below tau in some subdomain (Ritz values approach from above, so that count only
  // grows); the grown block starts from the current one, padded with fresh random columns.
  // A cluster of eigenvalues at the cut converges at the rate (lambda_w + s)/(lambda_m + s),
  // so the guard vectors matter.
  auto round8 = [](int v) { return std::min(MAXM, (v + 7) / 8 * 8); };
  const int mcap = fixed_count ? round8(mwant + 8) : round8(nev_max + 16);
  int m = fixed_count ? mcap : std::min(mcap, MSTART);
  std::vector<int64_t> voff;
  DevBuf<int64_t> d_voff, d_voff_prev;
  DevBuf<double> X, X_prev;
  int m_prev = 0;
  std::vector<double> lam_final;
  int it = 0;
  EventPair ev;
  c->mrhs_ms = c->mrhs_bytes = 0.0;
  c->mrhs_calls = 0;
  for (;;) {
  voff.assign(n_sub + 1, 0);
  for (int j = 0; j < n_sub; ++j) voff[j + 1] = voff[j] + 3 * sw.nD[j] * m;
  const int64_t tot = voff[n_sub];
  d_voff.alloc(n_sub + 1);
  to_dev(d_voff.p, voff.data(), n_sub + 1, s);
  X.alloc(tot);
  DevBuf<double> BX(tot), Y(tot), BY(tot), T(tot), MYb(m32 ? tot : 0);
  double* MY = m32 ? MYb.p : BX.p;                 // M Y (= B X for exact FP64 solves)
  DevBuf<int32_t> active(n_sub);
  std::vector<int32_t> act(n_sub, 1);
  to_dev(active.p, act.data(), n_sub, s);
  int64_t nch_max = 0;
  for (int j = 0; j < n_sub; ++j) nch_max = std::max(nch_max, (3 * sw.nD[j] + GCH - 1) / GCH);
  DevBuf<double> gpart((size_t)n_sub * nch_max * 2 * MAXM * MAXM), G((size_t)n_sub * 2 * MAXM * MAXM);
  DevBuf<double> Cm((size_t)n_sub * MAXM * MAXM), theta((size_t)n_sub * MAXM);
  DevBuf<double> rpart((size_t)n_sub * nch_max * 3 * MAXM), rsum((size_t)n_sub * 3 * MAXM);
  DevBuf<int> err(1);
  zero(err, s);
  const dim3 growD((unsigned)maxD, n_sub);
  const dim3 gvec(nblocks(3 * maxD * m, 256), n_sub);
  const dim3 grows(nblocks(3 * maxD, ROT_ROWS), n_sub);
  const dim3 gch((unsigned)nch_max, n_sub);
  hipLaunchKernelGGL(k_rand_init, gvec, dim3(256), 0, s, g, m, d_voff.p, X.p);
  if (m_prev)                                      // warm start: the previous block first
    hipLaunchKernelGGL(k_widen, dim3(nblocks(3 * maxD * m_prev, 256), n_sub), dim3(256), 0, s,
                       sw.d_nD.p, m_prev, d_voff_prev.p, X_prev.p, m, d_voff.p, X.p);
  X_prev.release();
  d_voff_prev.release();
  hipLaunchKernelGGL(k_bmul_rows, growD, dim3(64), 0, s, g, crow.p, cloc.p, cbv.p, m,
                     d_voff.p, active.p, X.p, BX.p);
  std::vector<double> h_theta((size_t)n_sub * MAXM), h_res((size_t)n_sub * 3 * MAXM);
  lam_final.assign((size_t)n_sub * MAXM, 0.0);
  int n_active = n_sub;
  bool grow = false;
  for (int itm = 0; itm < maxit && n_active > 0; ++itm, ++it) {
    if (m32) {
      // FP32 factor solves T ~ M^-1 (T = S Mt^-1 S): first step Y = T BX, then the
      // preconditioned-residual step Y = X - T (M X - B X Theta) with FP64 residuals
      // (MX is in Y after the previous rotation); exact eigenpairs are fixed points
      if (itm == 0)
        hipLaunchKernelGGL(k_copy_active, gvec, dim3(256), 0, s, 3 * maxD * m, sw.d_nD.p, m,
                           d_voff.p, active.p, BX.p, T.p);
      else
        hipLaunchKernelGGL(k_res_block, gvec, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p,
                           active.p, theta.p, Y.p, BX.p, T.p);
      hipLaunchKernelGGL(k_scale_rows, gvec, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p,
                         d_doff.p, active.p, dM.p, T.p, T.p);
      GX_HIP(hipEventRecord(ev.a, s));
      band_solve(Mb, d_voff.p, T.p, s, m, active.p);
      GX_HIP(hipEventRecord(ev.b, s));
      hipLaunchKernelGGL(k_scale_rows, gvec, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p,
                         d_doff.p, active.p, dM.p, T.p, T.p);
      if (itm == 0)
        hipLaunchKernelGGL(k_copy_active, gvec, dim3(256), 0, s, 3 * maxD * m, sw.d_nD.p, m,
                           d_voff.p, active.p, T.p, Y.p);
      else
        hipLaunchKernelGGL(k_sub_block, gvec, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p,
                           active.p, X.p, T.p, Y.p);
    } else {
      hipLaunchKernelGGL(k_copy_active, gvec, dim3(256), 0, s, 3 * maxD * m, sw.d_nD.p, m,
                         d_voff.p, active.p, BX.p, Y.p);
      GX_HIP(hipEventRecord(ev.a, s));
      band_solve(Mb, d_voff.p, Y.p, s, m, active.p);
      GX_HIP(hipEventRecord(ev.b, s));
    }
    hipLaunchKernelGGL(k_bmul_rows, growD, dim3(64), 0, s, g, crow.p, cloc.p, cbv.p, m,
                       d_voff.p, active.p, Y.p, BY.p);
    if (m32)
      hipLaunchKernelGGL(k_amul_rows, growD, dim3(64), 0, s, g, crowA.p, clocA.p, cbvA.p, m,
                         d_voff.p, active.p, Y.p, BY.p, sigma, MY);
    hipLaunchKernelGGL(k_gram, gch, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p, active.p, Y.p,
                       MY, BY.p, nch_max, gpart.p);
    hipLaunchKernelGGL(k_gram_sum, dim3(nblocks(2 * MAXM * MAXM, 256), n_sub), dim3(256), 0,
                       s, sw.d_nD.p, m, active.p, nch_max, gpart.p, G.p);
    hipLaunchKernelGGL(k_rayleigh_ritz, dim3(n_sub), dim3(256), 0, s, m, active.p, G.p, Cm.p,
                       theta.p, err.p);
    hipLaunchKernelGGL(k_rotate, grows, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p, active.p,
                       Cm.p, Y.p, T.p);             // new X
    hipLaunchKernelGGL(k_rotate, grows, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p, active.p,
                       Cm.p, MY, Y.p);              // M X_new
    hipLaunchKernelGGL(k_rotate, grows, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p, active.p,
                       Cm.p, BY.p, BX.p);           // B X_new
    hipLaunchKernelGGL(k_resid, gch, dim3(256), 0, s, sw.d_nD.p, m, d_voff.p, active.p,
                       theta.p, Y.p, BX.p, T.p, nch_max, rpart.p);
    hipLaunchKernelGGL(k_resid_sum, dim3(n_sub), dim3(3 * MAXM), 0, s, sw.d_nD.p, active.p,
                       nch_max, rpart.p, rsum.p);
    // new X into X for the active subdomains
    hipLaunchKernelGGL(k_copy_active, gvec, dim3(256), 0, s, 3 * maxD * m, sw.d_nD.p, m,
                       d_voff.p, active.p, T.p, X.p);
    GX_HIP(hipGetLastError());
    to_host(h_theta.data(), theta.p, h_theta.size(), s);
    to_host(h_res.data(), rsum.p, h_res.size(), s);
    c->mrhs_ms += ev.ms();
    c->mrhs_bytes += band_solve_bytes(Mb, m, act.data());
    ++c->mrhs_calls;
    int herr = 0;
    to_host(&herr, err.p, 1, s);
    if (herr) throw Error(GX_ENOCONV, "GenEO eigensolver: basis lost rank");
    band_solve_check(Mb, s);
    for (int j = 0; j < n_sub; ++j) {
      if (!act[j]) continue;
      // wanted pairs: the fixed count, or those below 1.5 tau (the test margin)
      int w = 0;
      if (fixed_count) {
        w = want[j];
      } else {
        // the pairs below tau, and the first one above it unless the cap nev_max is
        // reached (Ritz values approach the eigenvalues from above, so the count below tau
        // can only grow while iterating)
        while (w < m - 2 && h_theta[j * MAXM + w] - sigma < tau) ++w;
        if (m < mcap && w > m - 8) grow = true;
        w = std::min({w + 1, nev_max, m - 2});
      }
      // backward-error test: ||M x - theta B x|| <= tol * S ||x||, S = max over the block of
      // ||M x|| / ||x|| (an estimate of ||M||).  Relative to ||M x|| alone the test cannot
      // pass for rigid-body modes, whose M x = sigma B x is tiny: rounding sets the floor.
      const double* rj = h_res.data() + (size_t)j * 3 * MAXM;
      double S = 0.0;
      for (int a = 0; a < m; ++a)
        if (rj[2 * MAXM + a] > 0.0) S = std::max(S, std::sqrt(rj[MAXM + a] / rj[2 * MAXM + a]));
      bool ok = true;
      for (int a = 0; a < w; ++a)
        if (!(std::sqrt(rj[a]) <= tol * S * std::sqrt(rj[2 * MAXM + a]))) ok = false;
      if (ok) {
        act[j] = 0;
        --n_active;
        for (int a = 0; a < m; ++a) lam_final[j * MAXM + a] = h_theta[j * MAXM + a] - sigma;
      }
    }
    if (grow) break;
    to_dev(active.p, act.data(), n_sub, s);
  }
  if (grow) {                                      // wider block, warm-started from this one
    X_prev = std::move(X);
    d_voff_prev = std::move(d_voff);
    m_prev = m;
    m = mcap;
    continue;
  }
  if (n_active > 0)
    throw Error(GX_ENOCONV, "GenEO eigensolver did not converge in " + std::to_string(maxit) +
                                " iterations");
  break;
  }
  // selection
  sw.nev.assign(n_sub, 0);
  sw.lam.assign(n_sub, {});
  for (int j = 0; j < n_sub; ++j) {
    int k = 0;
    if (fixed_count)
      k = want[j];
    else
      while (k < nev_max && k < m - 2 && lam_final[j * MAXM + k] < tau) ++k;
    sw.nev[j] = k;
    for (int a = 0; a < k; ++a) sw.lam[j].push_back(lam_final[j * MAXM + a]);
  }
  c->phase_ms[3] = te.ms();
  c->eig_iters = it;
  Timer tc(s);
  // coarse basis Z_j (column-major on I_j) and K_0
  sw.c_off.assign(n_sub + 1, 0);
  sw.z_off.assign(n_sub + 1, 0);
  for (int j = 0; j < n_sub; ++j) {
    sw.c_off[j + 1] = sw.c_off[j] + sw.nev[j];
    sw.z_off[j + 1] = sw.z_off[j] + 3 * sw.nI[j] * sw.nev[j];
  }
  sw.n0 = sw.c_off[n_sub];
  if (sw.n0 == 0) {
    sw.two_level = false;
    c->phase_ms[4] = tc.ms();
    return;
  }
  sw.d_nev.alloc(n_sub);
  sw.d_c_off.alloc(n_sub + 1);
  sw.d_z_off.alloc(n_sub + 1);
  to_dev(sw.d_nev.p, sw.nev.data(), n_sub, s);
  to_dev(sw.d_c_off.p, sw.c_off.data(), n_sub + 1, s);
  to_dev(sw.d_z_off.p, sw.z_off.data(), n_sub + 1, s);
  sw.Z.alloc(std::max<int64_t>(sw.z_off[n_sub], 1));
  CoarseDev cd{sw.I_nodes.p, sw.d_offI.p, sw.d_nI.p, sw.d_z_off.p, sw.d_nev.p, sw.d_c_off.p};
  int64_t maxI = 0;
  for (int j = 0; j < n_sub; ++j) maxI = std::max(maxI, sw.nI[j]);
  hipLaunchKernelGGL(k_build_Z, dim3(nblocks(3 * maxI, 256), n_sub), dim3(256), 0, s, g, cd, m,
                     d_voff.p, X.p, sw.Z.p);
  std::vector<int64_t> vco(n_sub + 1, 0);
  for (int j = 0; j < n_sub; ++j) vco[j + 1] = vco[j] + 3 * sw.nD[j] * sw.nev[j];
  DevBuf<int64_t> d_vco(n_sub + 1);
  to_dev(d_vco.p, vco.data(), n_sub + 1, s);
  DevBuf<double> Vc(std::max<int64_t>(vco[n_sub], 1));
  hipLaunchKernelGGL(k_coarse_V, dim3((unsigned)maxD, n_sub), dim3(64), 0, s, g, cd,
                     c->row_ptr.p, c->col.p,
                     c->val.p, sw.Z.p, d_vco.p, Vc.p);
  DevBuf<int32_t> adj((size_t)n_sub * n_sub);
  zero(adj, s);
  hipLaunchKernelGGL(k_pair_adjacency, dim3(nblocks(N, 256)), dim3(256), 0, s, sw.node_and.p,
                     sw.node_or.p, sw.W, N, n_sub, adj.p);
  const int64_t n0 = sw.n0;
  DevBuf<double> K0(n0 * n0);
  zero(K0, s);
  hipLaunchKernelGGL(k_coarse_pair, dim3(n_sub, n_sub), dim3(256), 0, s, g, cd, n_sub, adj.p,
                     sw.Z.p, Vc.p, d_vco.p, n0, K0.p);
  band_layout(sw.C, {n0}, {n0 - 1}, false, s);
  sw.C.coarse = true;
  zero(sw.C.v64, s);
  hipLaunchKernelGGL(k_coarse_fill, dim3(nblocks(n0 * n0, 256)), dim3(256), 0, s, n0, K0.p,
                     sw.C.B[0], sw.C.ld[0], sw.C.v64.p);
  GX_HIP(hipGetLastError());
  band_factor(sw.C, s, "the coarse matrix K0 (near-dependent coarse vectors?)");
  const int64_t zero64 = 0;
  sw.d_c_xoff.alloc(1);
  to_dev(sw.d_c_xoff.p, &zero64, 1, s);
  const int64_t nchr = (3 * maxI + 1023) / 1024;
  sw.y0.alloc(n0);
  sw.y0part.alloc(n0 * nchr);
  GX_HIP(hipStreamSynchronize(s));
  c->phase_ms[4] = tc.ms();
}

}  // namespace gx

using namespace gx;

extern "C" {

// A stream of the set-up's own (default priority), drained before it goes.
struct SideStream {
  hipStream_t st = nullptr;
  SideStream() { GX_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking)); }
  ~SideStream() {
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  }
  SideStream(const SideStream&) = delete;
  SideStream& operator=(const SideStream&) = delete;
};

gx_status gx_geneo_setup(gx_ctx* c, const gx_geneo_opts* o, int32_t* nev_out,
                         int64_t* n0_out) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "gx_assemble has not been called");
  if (c->matrix_only) throw Error(GX_ESTATE, "needs an assembled mesh, not a loaded matrix");
  GX_REQUIRE(o && o->elem_part, "null options");
  GX_REQUIRE(o->n_sub >= 1 && o->n_sub <= 4096, "n_sub out of range");
  GX_REQUIRE(o->overlap >= 1 && o->overlap <= 16, "overlap must be in [1, 16]");
  GX_REQUIRE(o->precision == GX_FP64 || o->precision == GX_MIXED, "bad precision");
  GX_REQUIRE(o->nev_max <= 32, "nev_max must be <= 32");
  c->setup_done = false;
  c->sw = Schwarz();
  c->fp64_fallbacks = 0;
  Timer t1(c->stream);
  dd_build(c, o->elem_part, o->n_sub, o->overlap);
  c->phase_ms[1] = t1.ms();
  c->phase_ms[3] = c->phase_ms[4] = 0;
  c->sw.two_level = o->coarse != 0;
  if (c->sw.two_level) {
    // The interior factorisation shares nothing with the eigensolves: it runs on a side
    // stream while they run on the context's stream (the two sets of factors are then
    // resident together).  Its matrices are laid out and filled first; its factorisation
    // starts once the eigensolver's factorisation is done, so that it runs beside the
    // eigensolver's iterations (bound by memory traffic), not beside the other
    // factorisation, and a host thread of the job enqueues its launches, so that this
    // thread goes on to the iterations at once.  The side stream is declared first, so the
    // job (which waits for its streams when it goes) is destroyed before it.
    SideStream side;
    InteriorJob job;
    EventPair ev;
    {
      StreamScope scope(side.st);
      GX_HIP(hipEventRecord(ev.a, side.st));
      interior_factors_prepare(c, o->precision, side.st, job);
    }
    auto start_interior = [&]() {
      StreamScope scope(side.st);
      interior_factors_launch(c, side.st, job, true);
    };
    geneo_coarse(c, o, start_interior);
    interior_factors_finish(c, job);                 // joins the launching thread
    GX_HIP(hipEventRecord(ev.b, side.st));
    c->phase_ms[2] = ev.ms();
  } else {
    Timer t2(c->stream);
    interior_factors(c, o->precision);
    c->phase_ms[2] = t2.ms();
  }
  if (nev_out)
    for (int j = 0; j < o->n_sub; ++j) nev_out[j] = c->sw.two_level ? c->sw.nev[j] : 0;
  if (n0_out) *n0_out = c->sw.two_level ? c->sw.n0 : 0;
  c->setup_done = true;
  GX_API_END(c)
}

gx_status gx_tune(gx_ctx* c, int32_t param, int64_t value) {
  GX_API_BEGIN(c)
  GX_REQUIRE(param >= 0 && param < 2, "unknown tuning parameter");
  GX_REQUIRE(value >= 0 && value <= 8, "value out of range");
  c->tune[param] = (int)value;
  if (c->setup_done) {                             // takes effect at the next solve
    c->sw.A.force_groups[param] = (int)value;
    c->sw.A.solve_groups[param] = 0;
  }
  GX_API_END(c)
}

gx_status gx_stats(gx_ctx* c, int64_t* out) {
  GX_API_BEGIN(c)
  GX_REQUIRE(out, "null output");
  out[0] = c->eig_iters;
  out[1] = c->pcg_iters;
  out[2] = c->sw.A.total;
  out[3] = c->neumann_entries;
  out[4] = c->fp64_fallbacks;
  GX_API_END(c)
}

gx_status gx_subdomain_info(gx_ctx* c, int64_t* ni, int64_t* nn, int64_t* hb) {
  GX_API_BEGIN(c)
  if (!c->setup_done) throw Error(GX_ESTATE, "gx_geneo_setup has not been called");
  for (int j = 0; j < c->sw.n_sub; ++j) {
    if (ni) ni[j] = 3 * c->sw.nI[j];
    if (nn) nn[j] = 3 * c->sw.nD[j];
    if (hb) hb[j] = c->sw.A.B[j];
  }
  GX_API_END(c)
}

gx_status gx_geneo_setup_batch(int32_t n, gx_ctx* const* ctxs, const gx_geneo_opts* const* opts,
                               int32_t concurrent, int32_t* const* nev_out, int64_t* n0_out,
                               int32_t* status_out) {
  if (n < 1 || !ctxs || !opts || concurrent < 1) return GX_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i] || !opts[i]) return GX_EINVAL;
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) return GX_EINVAL;    // one set-up per context
  }
  const int T = std::min<int>(concurrent, n);
  for (int i = 0; i < n; ++i) ctxs[i]->share = T;
  std::vector<gx_status> st(n, GX_OK);
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= n) return;
      st[i] = gx_geneo_setup(ctxs[i], opts[i], nev_out ? nev_out[i] : nullptr,
                             n0_out ? n0_out + i : nullptr);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < T; ++t) {
    try {
      pool.emplace_back(work);
    } catch (const std::exception&) {
      break;                                       // fewer threads: the rest run below
    }
  }
  work();
  for (std::thread& th : pool) th.join();
  gx_status first = GX_OK;
  for (int i = 0; i < n; ++i) {
    ctxs[i]->share = 1;
    if (status_out) status_out[i] = st[i];
    if (first == GX_OK) first = st[i];
  }
  return first;
}

gx_status gx_geneo_eigenvalues(gx_ctx* c, int32_t j, double* lam) {
  GX_API_BEGIN(c)
  if (!c->setup_done || !c->sw.two_level) throw Error(GX_ESTATE, "no coarse space");
  GX_REQUIRE(j >= 0 && j < c->sw.n_sub && lam, "bad subdomain index");
  for (size_t k = 0; k < c->sw.lam[j].size(); ++k) lam[k] = c->sw.lam[j][k];
  GX_API_END(c)
}

}  // extern "C"
