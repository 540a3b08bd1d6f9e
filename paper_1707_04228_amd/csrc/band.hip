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
// Factorisation: right-looking, block columns of NB taken GP at a time; one launch per
// group factors its panels (diagonal blocks, their inverses, kept for the solves, and the
// panel rows), and the trailing window is updated with 128x128 tiles.  Matrices of
// different size and bandwidth run in the same launches.
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
  const int64_t* eoff;                            // envelope tables by 64-row blocks
  const int64_t* fcb;
  const int64_t* lrb;
};

// ---- Factorisation: right-looking blocked Cholesky in groups of GP panels of NB columns.
// The columns of a group [k0, k0 + GP NB) are factored by two launches: k_chain for the
// group's own rows, k_far for the rows below them.  The update of the trailing window by
// the group's panels is split in two k_syrk_wide launches: the next group's columns (then
// that group's k_chain, on the same stream), and all further columns on a second stream,
// at the same time.
constexpr int GP = 4;                             // panels per group
constexpr int CT = 256;                           // threads of a panel work-group
constexpr int64_t SPIN_LIMIT = (int64_t)1 << 22;  // polls before a wait gives up

// Loads and stores of data handed between the work-groups of one launch: agent-scope
// relaxed atomics, which bypass the per-XCD caches, so a reader sees the writer's values
// without a cache flush or invalidate on either side.
template <class T>
__device__ inline T co_load(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline void co_store(T* p, T x) {
  __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Raises a block's flag to this launch's epoch once every thread's hand-over stores have
// completed (waited for per thread, then a barrier).
__device__ inline void chain_signal(int* f, int epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded poll of a flag (thread 0); a poll that gives up raises bit 2 of the error word,
// and polls stop early once that bit is up, so every wave still reaches the end of the
// kernel.
__device__ inline void chain_wait(const int* f, int epoch, int* err) {
  for (int64_t k = 0; k < SPIN_LIMIT; ++k) {
    if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= epoch) return;
    if ((k & 255) == 255 && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 2))
      return;
    __builtin_amdgcn_s_sleep(1);
  }
  atomicOr(err, 2);
}

template <class S>
struct Chunk;                                     // reduction chunk: KC columns, LDS stride KS
template <>
struct Chunk<double> {
  static constexpr int KC = 32, KS = 34;
};
template <>
struct Chunk<float> {
  static constexpr int KC = 64, KS = 68;
};

// One launch per group for the group's own rows.  Work-group (p, j, t) owns the 64 rows
// [c0 + 64 t, c0 + 64 t + 64) of panel p (columns [c0, c0 + 64), c0 = k0 + 64 p) of matrix
// j; t = 0 is the diagonal block; blocks below the group (p + t >= GP) are k_far's and only
// raise their flags.  Work-groups are numbered: panel 0's diagonal blocks (all matrices),
// then panel by panel and matrix by matrix the blocks t >= 1, with the next panel's
// diagonal block right after block t = 1 (the last one it needs), so that the next
// factorisation runs while the rest of the panel is dispatched.  A work-group takes its number from a counter of the
// launch when it starts, not from its position in the grid, so every wait is for a
// work-group that is already running: the launch cannot deadlock, whatever order the
// hardware dispatches its work-groups in and whatever else occupies the device.
//   1. The block is brought up to date by this group's earlier panels (the earlier groups'
//      updates are done before the launch): A -= L[rows][K] L[panel rows][K]^T, after
//      waiting for the work-groups that produced them, with the matrix instruction in the
//      factor's precision.
//   2. t = 0: Cholesky of the 64x64 block and the inverse of its factor by one wave, in
//      16-column blocks (step 2a below); the inverse is handed to the panel's other
//      work-groups and kept for the triangular solves.
//      t > 0: waits for the inverse and forms L[rows][panel] = A Li^T (FP64 instruction).
//   3. The flag of (p, j, t) is raised.
// A non-positive pivot raises bit 1 of the error word and is replaced by 1.
template <class T>
__global__ void __launch_bounds__(CT) k_chain(BandArgs a, T* v, int64_t k0, int NR, int n_mat,
                                              int* flags, int* ticket, int epoch, double* inv,
                                              T* dinv, const int64_t* boff, int* err) {
  typedef Mfma<T> MT;
  typedef typename MT::S S;
  constexpr int KC = Chunk<S>::KC, KS = Chunk<S>::KS;
  constexpr int RP = CT / KC;                    // rows staged per pass
  constexpr int PER = NB / RP;                   // staged entries per thread and operand
  __shared__ double D[NB][NB + 1];               // the block; the factor (t = 0)
  __shared__ double Li[NB][NB + 1];              // the inverse of the diagonal block
  __shared__ double Wd[NB / 16][16][17];         // inverses of the 16x16 diagonal blocks
  __shared__ double Tt[16][17];                  // one tile of the inverse's assembly
  static_assert(NB * KS * sizeof(S) <= sizeof(D), "staging fits in the block buffers");
  S* Pr = reinterpret_cast<S*>(&D[0][0]);        // staging of step 1 (aliases D and Li)
  S* Ps = reinterpret_cast<S*>(&Li[0][0]);
  int p, j, t;
  {
    __shared__ int tk;
    if (threadIdx.x == 0) tk = atomicAdd(ticket, 1);
    __syncthreads();
    int b = tk;
    if (b < n_mat || NR == 1) {                  // panel 0's diagonal blocks
      p = b / n_mat;
      j = b - p * n_mat;
      t = 0;
    } else {
      b -= n_mat;
      for (p = 0; p < GP; ++p) {                 // section of panel p
        const int m = NR - 1 + (p + 1 < GP);
        if (b < n_mat * m) break;
        b -= n_mat * m;
      }
      j = b / (NR - 1 + (p + 1 < GP));
      const int o = b - j * (NR - 1 + (p + 1 < GP));
      if (o == 0) {
        t = 1;
      } else if (p + 1 < GP && o == 1) {         // the next panel's diagonal block
        p += 1;
        t = 0;
      } else {
        t = p + 1 < GP ? o : o + 1;
      }
    }
  }
  const int tr = p + t;                          // row block, counted from k0
  const int NRT = NR + GP - 1;
  int* fj = flags + (int64_t)j * GP * NRT;       // flag of (q, j, row block b): fj[q NRT + b]
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  const int64_t c0 = k0 + (int64_t)NB * p, r0 = c0 + (int64_t)NB * t;
  // no entries, or rows below the group (k_far's): only the flag
  if (c0 >= n || r0 >= n || r0 > c0 + NB - 1 + B || tr >= GP) {
    if (threadIdx.x == 0) __hip_atomic_store(fj + p * NRT + tr, epoch, __ATOMIC_RELEASE,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  T* base = v + a.off[j];
  const int64_t rs = ld - 1;                     // entry (r, c) at r * rs + B + c
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = 32 * (w & 1), wc = 32 * (w >> 1);
  const int kc_t = threadIdx.x % KC, i0 = threadIdx.x / KC;
  // the block's entries, loaded now and used after step 1 (entries outside the matrix or
  // the band read as 0; the diagonal block keeps its lower triangle)
  const int nb = (int)min<int64_t>(NB, n - c0);  // columns of the panel inside the matrix
  double av[2][4][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int rl = wr + 16 * i + MT::row(q, lk), cl = wc + 16 * jj + li;
        const int64_t r = r0 + rl, c = c0 + cl;
        av[i][q][jj] = (r < n && cl < nb && c >= r - B && (t > 0 || cl <= rl))
                           ? (double)base[r * rs + B + c] : 0.0;
      }
  // 1. A -= L[rows][K] L[panel rows][K]^T over this group's earlier panels K = [k0, c0),
  // once the work-groups that produced them are done; the next chunk is fetched while
  // the current one is multiplied
  typename MT::V acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = typename MT::V{0, 0, 0, 0};
  if (p > 0) {
    if (threadIdx.x == 0)
      for (int q = 0; q < p; ++q) {               // blocks past a panel's reach have none
        if (tr - q < NR) chain_wait(fj + q * NRT + tr, epoch, err);
        if (p - q < NR) chain_wait(fj + q * NRT + p, epoch, err);
      }
    __syncthreads();
    // the first chunk with an entry inside the envelope of the block's rows
    const int64_t lo = max(r0 - B, a.fcb[a.eoff[j] + r0 / NB]);
    const int64_t kstart = lo > k0 ? k0 + (lo - k0) / KC * KC : k0;
    S xr[PER], xs[PER];
    // 32-bit terms relative to the block: row i of a block is inside the matrix if
    // i < lim, and panel column q (counted from k0) is inside the band of that row if
    // q - i >= lo; rows' band origins are 32-bit offsets from the matrix start
    const int lim_r = (int)min<int64_t>(n - r0, NB), lim_s = (int)min<int64_t>(n - c0, NB);
    const int lo_r = (int)(r0 - B - k0), lo_s = (int)(c0 - B - k0), qend = (int)(c0 - k0);
    const uint32_t or0 = (uint32_t)(min(r0 + i0, n - 1) * rs + B + k0 + kc_t);
    const uint32_t os0 = (uint32_t)(min(c0 + i0, n - 1) * rs + B + k0 + kc_t);
    const uint32_t ostep = (uint32_t)(RP * rs);
    auto fetch = [&](int64_t kc) {
      const int qq = (int)(kc - k0) + kc_t;
      const uint32_t kd = (uint32_t)(kc - k0);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int i = i0 + RP * u;
        const bool okr = qq < qend && i < lim_r && qq - i >= lo_r;
        const bool oks = qq < qend && i < lim_s && qq - i >= lo_s;
        xr[u] = okr ? (S)co_load(base + (or0 + u * ostep + kd)) : (S)0;
        xs[u] = oks ? (S)co_load(base + (os0 + u * ostep + kd)) : (S)0;
      }
    };
    if (kstart < c0) fetch(kstart);
    for (int64_t kc = kstart; kc < c0; kc += KC) {
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        Pr[(i0 + RP * u) * KS + kc_t] = xr[u];
        Ps[(i0 + RP * u) * KS + kc_t] = xs[u];
      }
      __syncthreads();
      if (kc + KC < c0) fetch(kc + KC);
#pragma unroll
      for (int k = 0; k < KC; k += 4) {
        S fa[2], fb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) fa[i] = Pr[(wr + 16 * i + li) * KS + k + lk];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) fb[jj] = Ps[(wc + 16 * jj + li) * KS + k + lk];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) acc[i][jj] = MT::mma(fa[i], fb[jj], acc[i][jj]);
      }
      __syncthreads();
    }
  }
  // the updated block into D
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int rl = wr + 16 * i + MT::row(q, lk), cl = wc + 16 * jj + li;
        double x = av[i][q][jj] - (double)acc[i][jj][q];
        if (t == 0 && rl == cl && rl >= nb) x = 1.0;       // padding of a short last panel
        D[rl][cl] = x;
      }
  __syncthreads();
  double* invj = inv + ((int64_t)j * GP + p) * NB * NB;
  if (t == 0) {
    // 2a. Cholesky of the diagonal block and its inverse, by wave 0 alone (no barriers), in
    // 16-column blocks: the 16x16 diagonal block is factored in registers (lane r holds
    // row r; pivots and column entries come from other lanes by reads of their registers)
    // and inverted by forward substitution (lane c: column c); the panel below it is
    // L = A W^T with W that inverse, and the trailing triangle takes -= L L^T, both as
    // 16x16 tiles on the FP64 matrix instruction.  The inverse of the 64x64 factor is then
    // built tile by tile: Li(i, i) = W_i, Li(i, j) = -W_i sum_{j <= k < i} L(i, k) Li(k, j).
    if (w == 0) {
      typedef Mfma<double> M64;
      const int r16 = lane & 15;
      for (int kb = 0; kb < 4; ++kb) {
        const int b0 = 16 * kb;
        double f[16], rdg[16];                     // rdg: reciprocals of the pivots
#pragma unroll
        for (int c = 0; c < 16; ++c) f[c] = c <= r16 ? D[b0 + r16][b0 + c] : 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const double dii = lane_value(f[i], i);
          const bool ok = dii > 0.0;
          if (!ok && lane == 0) atomicOr(err, 1);
          // 1 / sqrt(dii): the hardware estimate, then two Newton steps
          // r <- r (3 - dii r^2) / 2, which bring it to full FP64 precision
          double r = 1.0;
          if (ok) {
            r = __builtin_amdgcn_rsq(dii);
            r = r * (1.5 - 0.5 * dii * r * r);
            r = r * (1.5 - 0.5 * dii * r * r);
          }
          rdg[i] = r;
          f[i] = r16 == i ? (ok ? dii * r : 1.0) : f[i] * r;
#pragma unroll
          for (int s2 = i + 1; s2 < 16; ++s2) f[s2] -= f[i] * lane_value(f[i], s2);
        }
        if (lane < 16)
#pragma unroll
          for (int c = 0; c < 16; ++c) D[b0 + r16][b0 + c] = c <= r16 ? f[c] : 0.0;
        double xi[16];                             // column r16 of the block's inverse
        // (the factor's entries L(i, k) are read back from LDS, the same address in every
        // lane, rather than from lane i's registers: they do not depend on xi, so the
        // reads are issued ahead, and they take no scalar registers)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          double sum = i == r16 ? 1.0 : 0.0;
#pragma unroll
          for (int k = 0; k < i; ++k) sum -= D[b0 + i][b0 + k] * xi[k];
          xi[i] = sum * rdg[i];
        }
        if (lane < 16)
#pragma unroll
          for (int i = 0; i < 16; ++i) Wd[kb][i][r16] = xi[i];
        for (int ti = kb + 1; ti < 4; ++ti) {      // panel tiles: L = A W^T
          v4d acc = v4d{0, 0, 0, 0};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            acc = M64::mma(D[16 * ti + li][b0 + 4 * ks + lk], Wd[kb][li][4 * ks + lk], acc);
#pragma unroll
          for (int q = 0; q < 4; ++q) D[16 * ti + M64::row(q, lk)][b0 + li] = acc[q];
        }
        for (int tj = kb + 1; tj < 4; ++tj)        // trailing tiles: -= L L^T
          for (int ti = tj; ti < 4; ++ti) {
            v4d acc = v4d{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
              acc = M64::mma(D[16 * ti + li][b0 + 4 * ks + lk], D[16 * tj + li][b0 + 4 * ks + lk],
                             acc);
#pragma unroll
            for (int q = 0; q < 4; ++q) D[16 * ti + M64::row(q, lk)][16 * tj + li] -= acc[q];
          }
      }
      // Li is assembled below the diagonal tiles only: its diagonal tiles are the W_i (read
      // from Wd) and it is zero above them
      for (int dd = 1; dd < 4; ++dd)
        for (int ti = dd; ti < 4; ++ti) {
          const int tj = ti - dd;
          v4d acc = v4d{0, 0, 0, 0};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)              // kt = tj: Li(tj, tj) = W_tj
            acc = M64::mma(D[16 * ti + li][16 * tj + 4 * ks + lk], Wd[tj][4 * ks + lk][li], acc);
          for (int kt = tj + 1; kt < ti; ++kt)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
              acc = M64::mma(D[16 * ti + li][16 * kt + 4 * ks + lk],
                             Li[16 * kt + 4 * ks + lk][16 * tj + li], acc);
#pragma unroll
          for (int q = 0; q < 4; ++q) Tt[M64::row(q, lk)][li] = acc[q];
          v4d o = v4d{0, 0, 0, 0};
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            o = M64::mma(Wd[ti][li][4 * ks + lk], Tt[4 * ks + lk][li], o);
#pragma unroll
          for (int q = 0; q < 4; ++q) Li[16 * ti + M64::row(q, lk)][16 * tj + li] = -o[q];
        }
    }
    __syncthreads();
    T* dj = dinv + boff[j] + (c0 / NB) * NB * NB;
    for (int idx = threadIdx.x; idx < NB * NB; idx += CT) {
      const int i = idx / NB, l = idx % NB;
      const double lv = (i >> 4) > (l >> 4)    ? Li[i][l]
                        : (i >> 4) == (l >> 4) ? Wd[i >> 4][i & 15][l & 15]
                                               : 0.0;
      co_store(invj + idx, lv);
      dj[idx] = (T)lv;
      if (i < nb && l <= i && i - l <= B) base[(c0 + i) * rs + B + c0 + l] = (T)D[i][l];
    }
  } else {
    // 2b. L[rows][panel] = A Li^T with the inverse of the diagonal block
    if (threadIdx.x == 0) chain_wait(fj + p * NRT + p, epoch, err);
    __syncthreads();
    {
      double lv[NB * NB / CT];                   // all loads issued before any is used
#pragma unroll
      for (int u = 0; u < NB * NB / CT; ++u) lv[u] = co_load(invj + threadIdx.x + CT * u);
#pragma unroll
      for (int u = 0; u < NB * NB / CT; ++u) {
        const int idx = threadIdx.x + CT * u;
        Li[idx / NB][idx % NB] = lv[u];
      }
    }
    __syncthreads();
    v4d x[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) x[i][jj] = v4d{0, 0, 0, 0};
#pragma unroll 4
    for (int k = 0; k < NB; k += 4) {
      double fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = D[wr + 16 * i + li][k + lk];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) fb[jj] = Li[wc + 16 * jj + li][k + lk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) x[i][jj] = Mfma<double>::mma(fa[i], fb[jj], x[i][jj]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int rl = wr + 16 * i + Mfma<double>::row(q, lk), cl = wc + 16 * jj + li;
          const int64_t r = r0 + rl, c = c0 + cl;
          if (r < n && cl < nb && c >= r - B) co_store(base + r * rs + B + c, (T)x[i][jj][q]);
        }
  }
  // 3.
  chain_signal(fj + p * NRT + tr, epoch);
}

// The rows below a group (row blocks GP, GP + 1, .. counted from k0) for all of the
// group's panels, once k_chain has factored the group's own rows: work-group (j, f) owns
// the 64 rows [k0 + 64 (GP + f), + 64) of matrix j and takes the panels in turn, each as
// k_chain's steps 1 and 2 for a block t > 0 - the update by the group's earlier panels
// (from its own results and the group's rows), then the product with the inverse of the
// panel's diagonal block.  Everything it reads was written by earlier launches or by
// itself, so nothing is waited for and plain loads suffice; the products are the same,
// in the same order, as k_chain's.
template <class T>
__global__ void __launch_bounds__(CT, 2) k_far(BandArgs a, T* v, int64_t k0, int NF, int n_mat,
                                               const double* inv) {
  typedef Mfma<T> MT;
  typedef typename MT::S S;
  constexpr int KC = Chunk<S>::KC, KS = Chunk<S>::KS;
  constexpr int VW = 16 / sizeof(S);             // entries per 16-byte load
  typedef S SV __attribute__((ext_vector_type(VW)));
  constexpr int RP = CT / (KC / VW);             // rows staged per pass
  constexpr int PER = NB / RP;                   // 16-byte loads per thread and operand
  __shared__ __attribute__((aligned(16))) double D[NB][NB + 1];    // the block
  __shared__ __attribute__((aligned(16))) double Li[NB][NB + 1];   // the inverse of the
                                                                   // panel's diagonal block
  static_assert(NB * KS * sizeof(S) <= sizeof(D), "staging fits in the block buffers");
  static_assert(KS * sizeof(S) % 16 == 0, "staged rows start on 16 bytes");
  S* Pr = reinterpret_cast<S*>(&D[0][0]);        // staging of the update (aliases D and Li)
  S* Ps = reinterpret_cast<S*>(&Li[0][0]);
  const int j = blockIdx.x / NF, f = blockIdx.x % NF;
  if (j >= n_mat) return;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  const int64_t r0 = k0 + (int64_t)NB * (GP + f);
  if (r0 >= n) return;
  T* base = v + a.off[j];
  const int64_t rs = ld - 1;                     // entry (r, c) at r * rs + B + c
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = 32 * (w & 1), wc = 32 * (w >> 1);
  const int kc_t = threadIdx.x % (KC / VW) * VW, i0 = threadIdx.x / (KC / VW);
#pragma unroll 1
  for (int p = 0; p < GP; ++p) {
    const int64_t c0 = k0 + (int64_t)NB * p;
    if (c0 >= n || r0 > c0 + NB - 1 + B) continue;   // no entries in this panel
    const int nb = (int)min<int64_t>(NB, n - c0);
    // the block's entries and the inverse of the panel's diagonal block are loaded first, so
    // that they arrive during the update
    T av[2][4][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int rl = wr + 16 * i + MT::row(q, lk), cl = wc + 16 * jj + li;
          const int64_t r = r0 + rl, c = c0 + cl;
          av[i][q][jj] = (r < n && cl < nb && c >= r - B) ? base[r * rs + B + c] : (T)0;
        }
    const double* invj = inv + ((int64_t)j * GP + p) * NB * NB;
    double lv[NB * NB / CT];
#pragma unroll
    for (int u = 0; u < NB * NB / CT; ++u) lv[u] = invj[threadIdx.x + CT * u];
    typename MT::V acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) acc[i][jj] = typename MT::V{0, 0, 0, 0};
    if (p > 0) {
      const int64_t lo = max(r0 - B, a.fcb[a.eoff[j] + r0 / NB]);
      const int64_t kstart = lo > k0 ? k0 + (lo - k0) / KC * KC : k0;
      // Each thread loads VW consecutive entries of a row at once (16 bytes: rows start on
      // 128-byte lines and k0 + (kc - k0) + kc_t is a multiple of VW, so the loads are
      // aligned).  The loads are unconditional: rows past the end of the matrix read at
      // most NB rows further, which the band allocation's padding covers, and entries
      // outside the band or the window are masked when they are staged.
      SV xr[PER], xs[PER];
      const int lim_r = (int)min<int64_t>(n - r0, NB), lim_s = (int)min<int64_t>(n - c0, NB);
      const int lo_r = (int)(r0 - B - k0), lo_s = (int)(c0 - B - k0), qend = (int)(c0 - k0);
      const uint32_t or0 = (uint32_t)((r0 + i0) * rs + B + k0 + kc_t);
      const uint32_t os0 = (uint32_t)((c0 + i0) * rs + B + k0 + kc_t);
      const uint32_t ostep = (uint32_t)(RP * rs);
      auto fetch = [&](int64_t kc) {
        const uint32_t kd = (uint32_t)(kc - k0);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          xr[u] = *reinterpret_cast<const SV*>(base + (or0 + u * ostep + kd));
          xs[u] = *reinterpret_cast<const SV*>(base + (os0 + u * ostep + kd));
        }
      };
      if (kstart < c0) fetch(kstart);
      for (int64_t kc = kstart; kc < c0; kc += KC) {
        const int qq = (int)(kc - k0) + kc_t;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int i = i0 + RP * u;
          SV wr_, ws_;
#pragma unroll
          for (int e = 0; e < VW; ++e) {
            const int q = qq + e;
            wr_[e] = (q < qend && i < lim_r && q - i >= lo_r) ? xr[u][e] : (S)0;
            ws_[e] = (q < qend && i < lim_s && q - i >= lo_s) ? xs[u][e] : (S)0;
          }
          *reinterpret_cast<SV*>(&Pr[i * KS + kc_t]) = wr_;
          *reinterpret_cast<SV*>(&Ps[i * KS + kc_t]) = ws_;
        }
        __syncthreads();
        if (kc + KC < c0) fetch(kc + KC);
#pragma unroll 4
        for (int k = 0; k < KC; k += 4) {
          S fa[2], fb[2];
#pragma unroll
          for (int i = 0; i < 2; ++i) fa[i] = Pr[(wr + 16 * i + li) * KS + k + lk];
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) fb[jj] = Ps[(wc + 16 * jj + li) * KS + k + lk];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) acc[i][jj] = MT::mma(fa[i], fb[jj], acc[i][jj]);
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int rl = wr + 16 * i + MT::row(q, lk), cl = wc + 16 * jj + li;
          D[rl][cl] = (double)av[i][q][jj] - (double)acc[i][jj][q];
        }
#pragma unroll
    for (int u = 0; u < NB * NB / CT; ++u) {
      const int idx = threadIdx.x + CT * u;
      Li[idx / NB][idx % NB] = lv[u];
    }
    __syncthreads();
    v4d x[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) x[i][jj] = v4d{0, 0, 0, 0};
#pragma unroll 4
    for (int k = 0; k < NB; k += 4) {
      double fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) fa[i] = D[wr + 16 * i + li][k + lk];
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) fb[jj] = Li[wc + 16 * jj + li][k + lk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) x[i][jj] = Mfma<double>::mma(fa[i], fb[jj], x[i][jj]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) {
          const int rl = wr + 16 * i + Mfma<double>::row(q, lk), cl = wc + 16 * jj + li;
          const int64_t r = r0 + rl, c = c0 + cl;
          if (r < n && cl < nb && c >= r - B) base[r * rs + B + c] = (T)x[i][jj][q];
        }
    // this panel's rows are read back by the next panel's update (other threads), and the
    // LDS buffers are restaged
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// The update of the trailing window by a group's panels, past the next group's columns,
// in 128 x 128 tiles of its lower triangle.  Eight waves each
// form a 64 x 32 eighth as 4 x 2 matrix-instruction tiles of 16 x 16, so six fragment reads
// from LDS feed eight instructions; two work-groups fit a compute unit.  The panels stream through LDS in chunks
// of KW columns (128 bytes of a row in FP64, 256 in FP32); the next chunk is loaded into registers while the
// current one is multiplied.  Chunks that lie left of the band for every row of the tile
// are skipped.  The LDS row stride (KW plus 2 doubles or 4 floats) spreads the 16 rows x 4
// reduction indices of one fragment read over distinct banks.
// The grid is one-dimensional over (matrix, tile) and consecutive tiles of a matrix go to
// the same XCD (work-groups are dealt round-robin to the eight XCDs), so a matrix's panels
// stay in that XCD's L2 while its tiles run.
constexpr int T2 = 128;                           // tile edge
constexpr int U2 = 512;                           // threads
template <class S>
struct Wide;
template <>
struct Wide<double> {
  static constexpr int KW = 16, KS = 18;
};
template <>
struct Wide<float> {
  static constexpr int KW = 64, KS = 68;
};

template <class T>
__device__ inline void wide_tile(BandArgs a, T* v, int64_t k0, int64_t kk, int64_t ts_lo,
                                 int64_t ts_hi, int64_t per_mat, int64_t lin) {
  typedef Mfma<T> MT;
  typedef typename MT::S S;
  constexpr int KW = Wide<S>::KW, KS = Wide<S>::KS;
  constexpr int VW = 16 / sizeof(S);             // entries per 16-byte load
  typedef S SV __attribute__((ext_vector_type(VW)));
  constexpr int RP = U2 / (KW / VW);             // rows staged per pass
  constexpr int PER = T2 / RP;                   // 16-byte loads per thread and operand
  __shared__ __attribute__((aligned(16))) S Pr[T2][KS];
  __shared__ __attribute__((aligned(16))) S Ps[T2][KS];
  const int j = (int)(lin / per_mat);
  const int64_t tile = lin - (int64_t)j * per_mat;
  const int64_t n = a.n[j], B = a.B[j], ld = a.ld[j];
  if (k0 >= n) return;
  const int64_t kj = min<int64_t>(kk, n - k0);
  const int64_t t0 = k0 + kj;
  const int64_t W = min<int64_t>(B, n - t0);
  if (W <= 0) return;
  const int64_t nt = (W + T2 - 1) / T2;
  const int64_t te = min(ts_hi, nt);
  int64_t ts, rem = tile;
  for (ts = ts_lo; ts < te && rem >= nt - ts; ++ts) rem -= nt - ts;
  if (ts >= te) return;
  const int64_t tr = ts + rem;
  T* base = v + a.off[j];
  const int64_t r0 = t0 + tr * T2, s0 = t0 + ts * T2, wend = t0 + W;
  const int64_t rs = ld - 1;                     // entry (r, c) at r * rs + B + c
  const int kc_t = threadIdx.x % (KW / VW) * VW, i0 = threadIdx.x / (KW / VW);
  // first chunk with an entry inside the envelope of the tile's rows (its two 64-row blocks)
  const int64_t* fcj = a.fcb + a.eoff[j];
  const int64_t b0 = r0 / NB;
  const int64_t fmin = b0 + 1 < (n + NB - 1) / NB ? min(fcj[b0], fcj[b0 + 1]) : fcj[b0];
  const int64_t lo = max(r0 - B, fmin) - k0;
  const int64_t kc_first = lo > 0 ? lo / KW * KW : 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = 64 * (w & 1), wc = 32 * (w >> 1);
  const bool idle = ts == tr && wc >= wr + 64;   // above the diagonal of a diagonal tile
  typename MT::V acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) acc[i][jj] = typename MT::V{0, 0, 0, 0};
  SV vr[PER], vs[PER];
  // 32-bit offsets from the matrix start (the host checks that they fit).  Rows past the
  // end of the matrix are not clamped: they read at most T2 rows further, which the band
  // allocation's padding covers, and are masked.  Each thread loads VW consecutive entries
  // of a row at once: rows start on 128-byte lines and k0 + kc + kc_t is a multiple of VW,
  // so every load is 16-byte aligned.
  const uint32_t ostep = (uint32_t)(RP * rs);
  const uint32_t or0 = (uint32_t)((r0 + i0) * rs + B + k0 + kc_t);
  const uint32_t os0 = (uint32_t)((s0 + i0) * rs + B + k0 + kc_t);
  auto load = [&](int64_t kc) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      vr[u] = *reinterpret_cast<const SV*>(base + (or0 + u * ostep + (uint32_t)kc));
      vs[u] = *reinterpret_cast<const SV*>(base + (os0 + u * ostep + (uint32_t)kc));
    }
  };

  // masks in 32-bit tile-relative terms: row i of a block is inside the window if
  // i < lim, and panel column q (0-based in the group) is inside the band of that row if
  // q - i >= lo (the block's first row starts the band at panel column lo)
  const int lim_r = (int)min<int64_t>(wend - r0, T2), lim_s = (int)min<int64_t>(wend - s0, T2);
  const int lo_r = (int)(r0 - B - k0), lo_s = (int)(s0 - B - k0);
  const int kjn = (int)kj;
  auto stage = [&](int64_t kc) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = i0 + RP * u;
      SV wr_, ws_;
#pragma unroll
      for (int e = 0; e < VW; ++e) {
        const int q = (int)kc + kc_t + e;
        wr_[e] = (q < kjn && i < lim_r && q - i >= lo_r) ? vr[u][e] : (S)0;
        ws_[e] = (q < kjn && i < lim_s && q - i >= lo_s) ? vs[u][e] : (S)0;
      }
      *reinterpret_cast<SV*>(&Pr[i][kc_t]) = wr_;
      *reinterpret_cast<SV*>(&Ps[i][kc_t]) = ws_;
    }
  };
  if (kc_first < kj) load(kc_first);
  for (int64_t kc = kc_first; kc < kj; kc += KW) {
    stage(kc);
    __syncthreads();
    if (kc + KW < kj) load(kc + KW);              // in flight during the products below
    if (!idle) {
#pragma unroll 1
      for (int k = 0; k < KW; k += 4) {
        S fa[4], fb[2];
#pragma unroll
        for (int i = 0; i < 4; ++i) fa[i] = Pr[wr + 16 * i + li][k + lk];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj) fb[jj] = Ps[wc + 16 * jj + li][k + lk];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) acc[i][jj] = MT::mma(fa[i], fb[jj], acc[i][jj]);
      }
    }
    __syncthreads();
  }
  if (idle) return;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + wr + 16 * i + MT::row(q, lk);
      if (r >= wend) continue;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj) {
        const int64_t s = s0 + wc + 16 * jj + li;
        if (s <= r) {
          T* e = base + r * ld + (s - r + B);
          *e = (T)((S)*e - acc[i][jj][q]);
        }
      }
    }
}

// One tile per work-group: work-group b runs on XCD x = b mod 8 and takes the (b / 8)-th
// tile of that XCD's consecutive share.
template <class T>
__global__ void __launch_bounds__(U2, 4) k_syrk_wide(BandArgs a, T* v, int64_t k0, int64_t kk,
                                                  int64_t ts_lo, int64_t ts_hi,
                                                  int64_t per_mat, int64_t total) {
  const int64_t x = blockIdx.x & 7, q = total >> 3, rem = total & 7;
  wide_tile<T>(a, v, k0, kk, ts_lo, ts_hi, per_mat, x * q + min(x, rem) + (blockIdx.x >> 3));
}

// Number of tiles k_syrk_wide enumerates per matrix for 128-column tile columns [lo, hi).
static int64_t wide_tiles(int64_t max_B, int64_t lo, int64_t hi) {
  const int64_t nt = (max_B + T2 - 1) / T2;
  int64_t c = 0;
  for (int64_t ts = lo; ts < std::min(hi, nt); ++ts) c += nt - ts;
  return c;
}


template <class T>
void band_factor_t(BandSet& bs, T* v, T* dinv, hipStream_t st, FactorJob& job, bool threaded) {
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p, bs.d_eoff.p, bs.d_fcb.p, bs.d_lrb.p};
  static_assert(GP * NB % T2 == 0, "a group spans whole wide tile columns");
  constexpr int64_t NEXT_TS = GP * NB / T2;              // tile columns of the next group
  for (int j = 0; j < bs.n_mat; ++j)
    GX_REQUIRE((bs.n[j] + T2) * bs.ld[j] + 64 < ((int64_t)1 << 31),
               "a band matrix of 2^31 entries or more exceeds the update's 32-bit offsets");
  const int NR = (int)((bs.max_B + NB - 1) / NB) + 1;   // row blocks of a panel
  // k_chain takes the group's own rows (GP row blocks per panel, those below the group
  // exit at once), k_far the NF row blocks below the group
  const int NRC = GP, NRT = NRC + GP - 1, NF = NR - 1;
  job.inv.alloc((size_t)bs.n_mat * GP * NB * NB);
  const int64_t n_groups = (bs.max_n + GP * NB - 1) / (GP * NB);
  job.flags.alloc((size_t)bs.n_mat * GP * NRT + n_groups);   // then one ticket counter per launch
  zero(job.flags, st);
  int* tickets = job.flags.p + (int64_t)bs.n_mat * GP * NRT;
  const int64_t nt2 = (bs.max_B + T2 - 1) / T2;
  const int64_t per_rest = wide_tiles(bs.max_B, NEXT_TS, nt2), tot_rest = per_rest * bs.n_mat;
  const int64_t per_next = wide_tiles(bs.max_B, 0, NEXT_TS), tot_next = per_next * bs.n_mat;
  const unsigned chain_blocks = (unsigned)((int64_t)GP * bs.n_mat * NRC);
  const unsigned far_blocks = (unsigned)((int64_t)bs.n_mat * NF);
  // group g on st: the update of its columns by group g - 1 (after the update of the same
  // columns by group g - 2, which ran on the second stream), then its k_chain and k_far;
  // then the update of the columns from group g + 2 on by its panels on the second stream,
  // at the same time as group g + 1's work on st.
  GX_HIP(hipStreamCreateWithFlags(&job.la, hipStreamNonBlocking));
  GX_HIP(hipEventCreateWithFlags(&job.chain, hipEventDisableTiming));
  GX_HIP(hipEventCreateWithFlags(&job.rest[0], hipEventDisableTiming));
  GX_HIP(hipEventCreateWithFlags(&job.rest[1], hipEventDisableTiming));
  const int64_t max_n = bs.max_n, max_B = bs.max_B;
  const int n_mat = bs.n_mat;
  const int64_t* boff = bs.d_boff.p;
  int* flags = job.flags.p;
  double* inv = job.inv.p;
  int* err = job.err.p;
  hipStream_t la = job.la;
  hipEvent_t ev_chain = job.chain, ev_rest[2] = {job.rest[0], job.rest[1]};
  auto launches = [=]() {
    bool recorded[2] = {false, false};
    int g = 0;
    for (int64_t k0 = 0; k0 < max_n; k0 += GP * NB, ++g) {
      if (recorded[g % 2]) GX_HIP(hipStreamWaitEvent(st, ev_rest[g % 2], 0));
      if (g > 0 && max_B > 0)
        hipLaunchKernelGGL(k_syrk_wide<T>, dim3((unsigned)tot_next), dim3(U2), 0, st, a, v,
                           k0 - GP * NB, (int64_t)GP * NB, (int64_t)0, NEXT_TS, per_next,
                           tot_next);
      hipLaunchKernelGGL(k_chain<T>, dim3(chain_blocks), dim3(CT), 0, st, a, v, k0, NRC,
                         n_mat, flags, tickets + g, g + 1, inv, dinv, boff, err);
      if (far_blocks)
        hipLaunchKernelGGL(k_far<T>, dim3(far_blocks), dim3(CT), 0, st, a, v, k0, NF, n_mat,
                           (const double*)inv);
      if (tot_rest && k0 + GP * NB < max_n) {
        GX_HIP(hipEventRecord(ev_chain, st));
        GX_HIP(hipStreamWaitEvent(la, ev_chain, 0));
        hipLaunchKernelGGL(k_syrk_wide<T>, dim3((unsigned)tot_rest), dim3(U2), 0, la, a, v,
                           k0, (int64_t)GP * NB, NEXT_TS, nt2, per_rest, tot_rest);
        GX_HIP(hipEventRecord(ev_rest[g % 2], la));
        recorded[g % 2] = true;
      }
    }
    for (int q = 0; q < 2; ++q)
      if (recorded[q]) GX_HIP(hipStreamWaitEvent(st, ev_rest[q], 0));
    GX_HIP(hipGetLastError());
  };
  if (!threaded) {
    launches();
    return;
  }
  // The launches only enqueue work (no host wait, no allocation), so a thread of the job
  // may make them while the caller goes on; band_factor_finish and the job's destructor
  // join it, and an error it met is raised by band_factor_finish.
  int dev = 0;
  GX_HIP(hipGetDevice(&dev));
  job.launcher = std::thread([launches, dev, &job]() {
    try {
      GX_HIP(hipSetDevice(dev));
      launches();
    } catch (...) {
      job.launch_error = std::current_exception();
    }
  });
}

FactorJob::~FactorJob() {
  if (launcher.joinable()) launcher.join();
  if (st) (void)hipStreamSynchronize(st);         // nothing of the job may still run when
  if (la) (void)hipStreamSynchronize(la);         // its buffers are released
  if (chain) (void)hipEventDestroy(chain);
  for (hipEvent_t e : rest)
    if (e) (void)hipEventDestroy(e);
  if (la) (void)hipStreamDestroy(la);
}

void band_factor_start(BandSet& bs, hipStream_t st, FactorJob& job, const char* what,
                       bool threaded) {
  GX_REQUIRE(!job.st, "factorisation job already started");
  job.st = st;
  job.what = what;
  job.err.alloc(1);
  zero(job.err, st);
  if (bs.fp32)
    band_factor_t<float>(bs, bs.v32.p, bs.dinv32.p, st, job, threaded);
  else
    band_factor_t<double>(bs, bs.v64.p, bs.dinv64.p, st, job, threaded);
}

void band_factor_finish(FactorJob& job) {
  GX_REQUIRE(job.st, "factorisation job not started");
  if (job.launcher.joinable()) job.launcher.join();
  if (job.launch_error) std::rethrow_exception(job.launch_error);
  int h = 0;
  to_host(&h, job.err.p, 1, job.st);               // waits for all of the job
  if (h & 2)
    throw Error(GX_EHIP, "banded Cholesky factorisation of " + job.what +
                             ": a work-group timed out waiting for a panel block");
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
constexpr int64_t BAND_PAD = 1024;               // trailing entries of a band allocation

// zero entries after the last matrix: the solves read up to BAND_PAD past its end, the
// trailing update up to T2 rows
static int64_t band_pad(int64_t max_B) { return BAND_PAD + T2 * (max_B + 1); }

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

// the same in FP32 (the hand-over scratch of the FP32 many-right-hand-side solve): the
// marker is a signalling-NaN payload, which arithmetic never produces either
constexpr uint32_t YMARK32 = 0x7FA5C0DEu;
__device__ inline bool is_mark(float v) { return __float_as_uint(v) == YMARK32; }
__device__ inline float poll_load(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void hand_over(float* p, float v) {
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
// ld: factor from base, inverse diagonal blocks from dv, envelope tables fcb / lrb (by
// 64-row blocks), right-hand side x, scratch y, z.
template <class T>
__device__ __forceinline__ void band_solve_1_mat(int64_t n, int64_t B, int64_t ld,
                                                 const T* base, const T* dv,
                                                 const int64_t* fcb, const int64_t* lrb,
                                                 const double* x, double* y, double* z, int g,
                                                 int G, int* err) {
  __shared__ double acc[SB];
  __shared__ double part[SW][SB];
  __shared__ double xs[GMAX - 1][SB];               // polled solutions of blocks in flight
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nblk = (n + SB - 1) / SB;
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
    // envelope start, rounded down to a 128-byte line (rows start on one: see band_layout)
    constexpr int64_t LA = 128 / sizeof(T);
    const int64_t cstart = max(max<int64_t>(ifirst - B, 0), fcb[k]) / LA * LA;
    {
      // a lane loads V adjacent columns of a row at once (16 bytes: two FP64 or four FP32
      // entries; columns from a line start are multiples of V, so every load is aligned),
      // 64 V columns per step, 512 columns per pass
      constexpr int V = 16 / sizeof(T);
      constexpr int US = 512 / (64 * V);            // steps per pass
      typedef T TV __attribute__((ext_vector_type(V)));
      for (int64_t c0 = cstart + V * lane; c0 < done_end + V * lane; c0 += 64 * V * US) {
        TV l[US][RPW];
        double xv[US][V];
#pragma unroll
        for (int u = 0; u < US; ++u) {
          const int64_t cc = c0 + 64 * V * u;
#pragma unroll
          for (int e = 0; e < V; ++e) xv[u][e] = poll_load(y + min<int64_t>(cc + e, done_end - 1));
#pragma unroll
          for (int r = 0; r < RPW; ++r) l[u][r] = *reinterpret_cast<const TV*>(rp[r] + cc);
        }
#pragma unroll
        for (int u = 0; u < US; ++u) {
          const int64_t cc = c0 + 64 * V * u;
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const double xe = cc + e < done_end ? xv[u][e] : 0.0;
#pragma unroll
            for (int r = 0; r < RPW; ++r)
              s[r] += (double)l[u][r][e] * (cc + e >= ifirst + r - B ? xe : 0.0);
          }
        }
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
    const int64_t rend = min(min<int64_t>(n, i0 + nb + B), lrb[kb]);   // envelope end
    const int64_t kdone = kb + G;                  // row blocks >= kdone complete
    const int64_t done_beg = min<int64_t>(rend, kdone * SB);
    const int64_t cidx = i0 + lane;
    double sacc = 0.0;
    {
      // lane l loads the V adjacent columns from V (l mod 64 / V) of the rows
      // r0 + 8 (V v + l / (64 / V)) (16 bytes, aligned as above), so one load covers V
      // rows; the row groups' sums are then added and handed to the lanes of their columns
      constexpr int V = 16 / sizeof(T);
      constexpr int LPR = 64 / V;                   // lanes per row
      typedef T TV __attribute__((ext_vector_type(V)));
      const int pr = lane % LPR, hf = lane / LPR;
      const int64_t cv = i0 + V * pr;
      double sv[V];
#pragma unroll
      for (int e = 0; e < V; ++e) sv[e] = 0.0;
      for (int64_t r0 = done_beg + wave; r0 < rend; r0 += SW * UB) {
        TV l[UB / V];
        const double xz = poll_load(z + min<int64_t>(r0 + SW * (lane % UB), rend - 1));
#pragma unroll
        for (int v = 0; v < UB / V; ++v) {
          const int64_t rr = min<int64_t>(r0 + SW * (V * v + hf), rend - 1);
          l[v] = *reinterpret_cast<const TV*>(cb + rr * rs + cv);
        }
#pragma unroll
        for (int v = 0; v < UB / V; ++v) {
          const int64_t rr = r0 + SW * (V * v + hf);
          const double xu = __shfl(xz, V * v + hf);
#pragma unroll
          for (int e = 0; e < V; ++e)
            sv[e] += (double)l[v][e] * ((rr < rend && rr - B <= cv + e) ? xu : 0.0);
        }
      }
#pragma unroll
      for (int m = LPR; m < 64; m *= 2)
#pragma unroll
        for (int e = 0; e < V; ++e) sv[e] += __shfl_xor(sv[e], m);
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const double t = __shfl(sv[e], lane / V);
        if (lane % V == e) sacc = t;
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
  band_solve_1_mat<T>(n, B, ld, v + a.off[j], dinv + boff[j], a.fcb + a.eoff[j],
                      a.lrb + a.eoff[j], xall + xoff[j], yall + yoff[j], zall + yoff[j], g, G,
                      err);
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
                      static_cast<const T*>(t.dinv), t.fcb, t.lrb, t.x, t.y, t.z, g, (int)t.G,
                      err);
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
// (forward into y, backward into z, z copied into x afterwards), kept in the factor's
// precision (FP32 factors: FP32 scratch, half the bytes of the solution rows that every
// chunk reads): solution entries are loaded with agent-scope relaxed atomics, and a chunk
// is staged only once none of the entries it needs is a marker (a chunk still in flight
// is polled again until then).
constexpr int MC = 32;                            // right-hand sides per launch, at most
constexpr int MT = 512;                           // threads per work-group
constexpr int AL = SB * SB / MT;                  // band-chunk entries per thread (8)

template <class T, int M>
__global__ void __launch_bounds__(MT) k_band_solve_m(
    BandArgs a, const T* v, const T* dinv, const int64_t* boff, const int64_t* xoff,
    const double* xall, T* yall, T* zall, const int64_t* yoff, int G, int n_pad,
    int n_mat, const int32_t* active, int* err) {
  typedef Mfma<T> MF;
  typedef typename MF::S S;
  typedef T Y;                                    // hand-over scratch: the factor's precision
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
  const int64_t* fcb = a.fcb + a.eoff[j];
  const int64_t* lrb = a.lrb + a.eoff[j];
  const double* x = xall + xoff[j];
  Y* y = yall + yoff[j] * M;
  Y* z = zall + yoff[j] * M;
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
  auto fetch = [&](bool bwd, int64_t i0, int64_t kk, T (&fa)[AL], Y (&fy)[YL]) {
    const int64_t r0 = (bwd ? kk * SB : i0) + wave;
    const int64_t c = (bwd ? i0 : kk * SB) + lane;
#pragma unroll
    for (int u = 0; u < AL; ++u) fa[u] = cb[min<int64_t>(r0 + 8 * u, n - 1) * rs + c];
    const int64_t yend = min<int64_t>((int64_t)SB * M, (n - kk * SB) * M);   // rows < n
    const Y* xs = (bwd ? z : y) + kk * SB * M;
#pragma unroll
    for (int u = 0; u < YL; ++u) fy[u] = poll_load(xs + min<int64_t>(threadIdx.x + MT * u, yend - 1));
  };
  auto stage = [&](int buf, bool bwd, int64_t i0, int nb, int64_t kk, const T (&fa)[AL],
                   Y (&fy)[YL]) {
    {                                              // until every needed entry is handed over
      const int64_t yend = min<int64_t>((int64_t)SB * M, (n - kk * SB) * M);
      const Y* xs = (bwd ? z : y) + kk * SB * M;
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
    Y fy0[YL], fy1[YL];
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
          const Y yb = poll_load(y + (i0 + min(ii, nb - 1)) * M + cc);
          bb[r] = (double)yb;
          ok = ok && (!tile || ii >= nb || !is_mark(yb));
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
    Y* dst = bwd ? z : y;
    if (tile)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ii = 16 * rt + MF::row(r, lk), col = 16 * ct + li;
        if (ii < nb && col < M) hand_over(dst + (i0 + ii) * M + col, (Y)yv[r]);
      }
    __syncthreads();
  };
  // ---- forward: chunks in increasing order; those from kdone on are still in flight
  for (int64_t k = g; k < nblk; k += G) {
    const int64_t i0 = k * SB;
    const int nb = (int)min<int64_t>(SB, n - i0);
    const int64_t kfirst = max(max<int64_t>(i0 - B, 0), fcb[k]) / SB;   // envelope start
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
    const int64_t klast = (min(min<int64_t>(n, i0 + nb + B), lrb[kb]) - 1) / SB;   // last row block
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

__global__ void k_fill_mark32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = __uint_as_float(YMARK32);
}

// z_j -> x_j for the active matrices (n_j rows of w columns)
template <class Y>
__global__ void k_copy_out_m(const int64_t* nrows, const int64_t* xoff, const int64_t* yoff,
                             int w, const Y* z, double* x, const int32_t* active) {
  const int j = blockIdx.y;
  if (active && !active[j]) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nrows[j] * w) x[xoff[j] + i] = (double)z[yoff[j] * w + i];
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
  const dim3 cgrid(nblocks(bs.max_n * M, 256), bs.n_mat);
  if (bs.fp32) {                                   // FP32 scratch in the same buffer
    float* y = reinterpret_cast<float*>(bs.mbuf.p);
    float* z = y + rows * M;
    hipLaunchKernelGGL(k_fill_mark32, dim3(nblocks(2 * rows * M, 256)), dim3(256), 0, st, y,
                       2 * rows * M);
    hipLaunchKernelGGL((k_band_solve_m<float, M>), dim3(G * n_pad), dim3(MT), 0, st, a, bs.v32.p,
                       bs.dinv32.p, bs.d_boff.p, d_xoff, x, y, z, bs.d_yoff.p, G, n_pad,
                       bs.n_mat, active, err);
    hipLaunchKernelGGL(k_copy_out_m<float>, cgrid, dim3(256), 0, st, bs.d_n.p, d_xoff,
                       bs.d_yoff.p, M, z, x, active);
  } else {
    double* y = bs.mbuf.p;
    double* z = bs.mbuf.p + rows * M;
    hipLaunchKernelGGL(k_fill_mark, dim3(nblocks(2 * rows * M, 256)), dim3(256), 0, st, y,
                       2 * rows * M);
    hipLaunchKernelGGL((k_band_solve_m<double, M>), dim3(G * n_pad), dim3(MT), 0, st, a,
                       bs.v64.p, bs.dinv64.p, bs.d_boff.p, d_xoff, x, y, z, bs.d_yoff.p, G,
                       n_pad, bs.n_mat, active, err);
    hipLaunchKernelGGL(k_copy_out_m<double>, cgrid, dim3(256), 0, st, bs.d_n.p, d_xoff,
                       bs.d_yoff.p, M, z, x, active);
  }
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
  BandArgs a{bs.d_n.p, bs.d_B.p, bs.d_ld.p, bs.d_off.p, bs.d_eoff.p, bs.d_fcb.p, bs.d_lrb.p};
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
      t.fcb = bs.d_fcb.p + bs.eoff[j];
      t.lrb = bs.d_lrb.p + bs.eoff[j];
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

// zero the entries between one matrix's storage and the next (the line alignment of the
// starts leaves up to A - 1 of them); the fills write only the matrices' own rows, and a
// load left of a row's band, masked by a factor 0, must not meet a NaN there
template <class T>
__global__ void k_zero_gaps(int n_mat, int A, const int64_t* off, const int64_t* nn,
                            const int64_t* ld, int64_t total, T* v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = i / A, k = i % A;
  if (j >= n_mat) return;
  const int64_t e = off[j] + nn[j] * ld[j] + k;
  const int64_t next = j + 1 < n_mat ? off[j + 1] : total;
  if (e < next) v[e] = (T)0;
}

void band_layout(BandSet& bs, const std::vector<int64_t>& n, const std::vector<int64_t>& B,
                 bool fp32, hipStream_t st, const std::vector<int32_t>* first_node) {
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
  // the stored half-bandwidth is B rounded up to a multiple of A, the entries of a 128-byte
  // line, and every matrix starts on a multiple of A: entry (r, c) then sits at an offset
  // congruent to c modulo A, so a row's entries from any multiple of A on fill whole
  // lines.  The extra band entries left of the band are zeros (outside the envelope).
  const int64_t A = fp32 ? 32 : 16;
  for (size_t j = 0; j < n.size(); ++j) {
    bs.B[j] = (B[j] + A - 1) / A * A;
    bs.ld[j] = bs.B[j] + 1;
    o = (o + A - 1) / A * A;
    bs.off[j] = o;
    o += n[j] * bs.ld[j];
    bs.max_n = std::max<int64_t>(bs.max_n, n[j]);
    bs.max_B = std::max<int64_t>(bs.max_B, bs.B[j]);
  }
  bs.total = o;
  // the envelope: row r from its first column f(r) (3 x its node's first coupled node, or
  // r - B) to the diagonal; env counts its entries, env_flops the Cholesky flops over it
  // (column c: h^2 + 2 h + 1 with h the rows below c that reach it), fcb / lrb its tables
  bs.eoff.assign(n.size() + 1, 0);
  for (size_t j = 0; j < n.size(); ++j) bs.eoff[j + 1] = bs.eoff[j] + (n[j] + SB - 1) / SB;
  std::vector<int64_t> fcb(std::max<int64_t>(bs.eoff[n.size()], 1)), lrb(fcb.size());
  bs.env.assign(n.size(), 0);
  bs.env_flops = 0.0;
  size_t node0 = 0;
  for (size_t j = 0; j < n.size(); ++j) {
    const int64_t nj = n[j], Bj = B[j], nbk = (nj + SB - 1) / SB;
    GX_REQUIRE(!first_node || (nj % 3 == 0 && node0 + nj / 3 <= first_node->size()),
               "band layout: a first node for every node of every matrix");
    int64_t* fj = fcb.data() + bs.eoff[j];
    int64_t* lj = lrb.data() + bs.eoff[j];
    std::vector<int64_t> reach(nbk, 0), diff(nj + 1, 0);
    for (int64_t b = 0; b < nbk; ++b) fj[b] = nj;
    for (int64_t r = 0; r < nj; ++r) {
      int64_t f = first_node ? 3 * (int64_t)(*first_node)[node0 + r / 3] : r - Bj;
      f = std::min(std::max(f, std::max<int64_t>(r - Bj, 0)), r);
      fj[r / SB] = std::min(fj[r / SB], f);
      reach[f / SB] = std::max(reach[f / SB], r + 1);
      bs.env[j] += r - f + 1;
      ++diff[f];
      --diff[r];
    }
    int64_t run = 0, h = 0;
    for (int64_t b = 0; b < nbk; ++b) {
      run = std::max(run, reach[b]);
      lj[b] = std::max(run, std::min(nj, (b + 1) * SB));
    }
    for (int64_t c = 0; c < nj; ++c) {
      h += diff[c];
      bs.env_flops += (double)h * h + 2.0 * h + 1.0;
    }
    if (first_node) node0 += nj / 3;
  }
  bs.d_eoff.alloc(n.size() + 1);
  bs.d_fcb.alloc(fcb.size());
  bs.d_lrb.alloc(lrb.size());
  to_dev(bs.d_eoff.p, bs.eoff.data(), n.size() + 1, st);
  to_dev(bs.d_fcb.p, fcb.data(), fcb.size(), st);
  to_dev(bs.d_lrb.p, lrb.data(), lrb.size(), st);
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
    bs.v32.alloc(o + band_pad(bs.max_B));
    GX_HIP(hipMemsetAsync(bs.v32.p + o, 0, band_pad(bs.max_B) * sizeof(float), st));
    hipLaunchKernelGGL(k_zero_gaps<float>, dim3(nblocks((int64_t)n.size() * A, 256)), dim3(256),
                       0, st, bs.n_mat, (int)A, bs.d_off.p, bs.d_n.p, bs.d_ld.p, o, bs.v32.p);
    bs.dinv32.alloc(bs.boff[n.size()]);
  } else {
    bs.v32.release();
    bs.dinv32.release();
    bs.v64.alloc(o + band_pad(bs.max_B));
    GX_HIP(hipMemsetAsync(bs.v64.p + o, 0, band_pad(bs.max_B) * sizeof(double), st));
    hipLaunchKernelGGL(k_zero_gaps<double>, dim3(nblocks((int64_t)n.size() * A, 256)), dim3(256),
                       0, st, bs.n_mat, (int)A, bs.d_off.p, bs.d_n.p, bs.d_ld.p, o, bs.v64.p);
    bs.dinv64.alloc(bs.boff[n.size()]);
  }
  bs.solve_groups[0] = bs.solve_groups[1] = 0;
  GX_HIP(hipStreamSynchronize(st));
}


// ---------------------------------------------------------------------------------------
// Stand-alone factor-and-solve of caller-supplied band matrices (exposed for testing the
// subdomain solver in isolation).
// caller band entry e (bandwidth bw[j], rows of bw[j] + 1 entries) into the set's storage
// (bandwidth sB[j], offsets soff[j]), which is zero beforehand
__global__ void k_band_import(int64_t total, const double* src, const double* dscale,
                              const int64_t* off, const int64_t* nn, const int64_t* bw,
                              const int64_t* doff, int n_mat, const int64_t* soff,
                              const int64_t* sB, float* d32, double* d64) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int j = 0;
  while (j + 1 < n_mat && off[j + 1] <= e) ++j;
  const int64_t B = bw[j], r = (e - off[j]) / (B + 1), c = r + (e - off[j]) % (B + 1) - B;
  if (c < 0) return;                               // left of the first column: none
  double v = src[e];
  if (dscale) v *= dscale[doff[j] + r] * dscale[doff[j] + c];
  const int64_t d = soff[j] + r * (sB[j] + 1) + (c - r + sB[j]);
  if (d32) d32[d] = (float)v;
  else d64[d] = v;
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
  if (fp32)
    zero(bs.v32, s);
  else
    zero(bs.v64, s);
  DevBuf<int64_t> d_off(n_mat + 1), d_doff(n_mat + 1), d_xoff(n_mat), d_bw(n_mat);
  to_dev(d_off.p, off.data(), n_mat + 1, s);
  to_dev(d_bw.p, bv.data(), n_mat, s);
  to_dev(d_doff.p, doff.data(), n_mat + 1, s);
  to_dev(d_xoff.p, xoff.data(), n_mat, s);
  DevBuf<double> dsc;
  if (fp32) {
    dsc.alloc(doff[n_mat]);
    hipLaunchKernelGGL(k_band_diag, dim3(nblocks(doff[n_mat], 256)), dim3(256), 0, s,
                       doff[n_mat], band, d_off.p, bs.d_n.p, d_bw.p, d_doff.p, n_mat, dsc.p);
  }
  hipLaunchKernelGGL(k_band_import, dim3(nblocks(off[n_mat], 256)), dim3(256), 0, s,
                     off[n_mat], band, fp32 ? dsc.p : nullptr, d_off.p, bs.d_n.p, d_bw.p,
                     d_doff.p, n_mat, bs.d_off.p, bs.d_B.p, fp32 ? bs.v32.p : nullptr,
                     fp32 ? nullptr : bs.v64.p);
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
