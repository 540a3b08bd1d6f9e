// Internal declarations shared by the gx HIP sources (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <functional>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/gx.h"

struct gx_ctx;

namespace gx {

struct Error : std::runtime_error {
  gx_status code;
  Error(gx_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define GX_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::gx::Error(e_ == hipErrorOutOfMemory ? GX_ENOMEM : GX_EHIP,              \
                        std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

#define GX_REQUIRE(cond, msg)                                                         \
  do {                                                                                \
    if (!(cond)) throw ::gx::Error(GX_EINVAL, msg);                                   \
  } while (0)

// Debugging aid: with GX_POISON_ALLOC=1 in the environment every new floating-point device
// buffer is filled with a huge finite value (bytes 0x7F), so a kernel that uses memory
// nobody wrote shows up as a wildly wrong result; reads masked by a zero factor stay exact.
inline bool poison_alloc() {
  static const bool on = [] {
    const char* e = std::getenv("GX_POISON_ALLOC");
    return e && e[0] == '1';
  }();
  return on;
}

// Device memory for DevBuf, with a per-device cache of released blocks (hipFree
// synchronises the whole device, which would serialise contexts set up concurrently).  A
// block released during an API call on a context is tagged with that context, the stream
// its work went to (the context's, or a side stream, StreamScope) and an event recorded
// there: a request of the same context for the same stream takes the block back with no
// wait (stream order), and any other request waits on the host for the event (that
// stream's work up to the release, not the whole device).  Blocks released on an
// idle device (IdleScope, a destroyed context) need no wait; blocks released outside any
// context are reused after a device synchronisation.  Blocks of 64 MiB and more are cached
// up to three quarters of the device's memory (a large block released with no room left
// frees the large blocks released longest ago, after a device synchronisation), smaller
// tagged or idle blocks up to 1 GiB per device.  A failed hipMalloc empties the cache of
// that device and retries.  dev_forget(ctx) marks a context's blocks idle (its stream
// must have been synchronised).
void* dev_alloc(size_t bytes, int* dev, hipError_t* err);
void dev_free(void* p, size_t bytes, int dev);
void dev_forget(const gx_ctx* c);

// While one exists on a thread, the blocks that thread releases are marked idle.
struct IdleScope {
  bool prev;
  IdleScope();
  ~IdleScope();
  IdleScope(const IdleScope&) = delete;
  IdleScope& operator=(const IdleScope&) = delete;
};

// The context of the API call running on this thread (tags released device blocks); set
// for the duration of a call by GX_API_BEGIN.
struct CtxScope {
  gx_ctx* prev;
  hipStream_t prev_stream;
  explicit CtxScope(gx_ctx* c);
  ~CtxScope();
  CtxScope(const CtxScope&) = delete;
  CtxScope& operator=(const CtxScope&) = delete;
};

// While one exists on a thread, the context's work that the thread enqueues, and the blocks
// it releases, belong to stream s instead of the context's own stream (a side stream).
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s);
  ~StreamScope();
  StreamScope(const StreamScope&) = delete;
  StreamScope& operator=(const StreamScope&) = delete;
};

// Owning device buffer.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  int dev = -1;
  DevBuf() = default;
  explicit DevBuf(size_t count) { alloc(count); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), dev(o.dev) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      dev = o.dev;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) {
      hipError_t e = hipSuccess;
      p = static_cast<T*>(dev_alloc(count * sizeof(T), &dev, &e));
      if (!p) {
        n = 0;
        throw Error(GX_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) +
                                   " bytes failed: " + hipGetErrorString(e));
      }
      if (std::is_floating_point<T>::value && poison_alloc()) {
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMemset(p, 0x7F, count * sizeof(T)) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
          throw Error(GX_EHIP, "poisoning a new buffer failed");
      }
    }
  }
  void release() {
    if (p) dev_free(p, n * sizeof(T), dev);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  operator T*() const { return p; }
};

// Pinned host buffer (device-to-host copies that the host reads after a stream sync)
template <class T>
struct HostBuf {
  T* p = nullptr;
  HostBuf() = default;
  HostBuf(const HostBuf&) = delete;
  HostBuf& operator=(const HostBuf&) = delete;
  ~HostBuf() {
    if (p) (void)hipHostFree(p);
  }
  void alloc(size_t count) {
    if (p) return;
    GX_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), count * sizeof(T), hipHostMallocDefault));
  }
};


template <class T>
inline void zero(DevBuf<T>& b, hipStream_t s) {
  if (b.n) GX_HIP(hipMemsetAsync(b.p, 0, b.bytes(), s));
}
template <class T>
inline void to_dev(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) GX_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
inline void to_host(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) GX_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s));
  GX_HIP(hipStreamSynchronize(s));
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// v of lane l (l wave-uniform), through the scalar unit
__device__ inline double lane_value(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Exclusive prefix sum of n int64 values in place; returns the total.  tmp must hold
// scan_tmp_size(n) elements.
size_t scan_tmp_size(int64_t n);
int64_t exclusive_scan(int64_t* data, int64_t n, int64_t* tmp, hipStream_t s);
int64_t exclusive_scan32(int32_t* data, int64_t n, int64_t* tmp, hipStream_t s);

__device__ inline double wave_sum_d(double s) {
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

struct BandView {
  const int64_t* B;
  const int64_t* ld;
  const int64_t* off;
};

// ------------------------------------------------------------------------------------
// Decomposition and preconditioner state.
struct BandSet {
  // Banded lower factors of a batch of SPD matrices, row-major band storage:
  // entry (r, c), r - B <= c <= r, of matrix j lives at off[j] + r * ld[j] + (c - r + B).
  int n_mat = 0;
  std::vector<int64_t> n, B, ld, off;          // host copies
  // envelope (profile) entries of each matrix's lower triangle, diagonal included: the
  // entries from each row's first nonzero column to the diagonal (Cholesky creates no fill
  // outside it).  band_layout sets it to the band itself; callers that know the matrices'
  // profile replace it.
  std::vector<int64_t> env;
  double env_flops = 0.0;                      // Cholesky flops over the envelope
  // the envelope by 64-row blocks (block b of matrix j at eoff[j] + b): fcb, the first
  // column any row of the block reaches; lrb, one past the last row that reaches a column
  // of the block.  From each row's first column when band_layout is given it, otherwise
  // from the band.  The kernels skip the 64-column steps outside it (exact zeros: Cholesky
  // creates no fill outside the envelope).
  std::vector<int64_t> eoff;
  DevBuf<int64_t> d_eoff, d_fcb, d_lrb;
  DevBuf<int64_t> d_n, d_B, d_ld, d_off;       // device copies
  int64_t total = 0;                           // stored entries
  int max_n = 0, max_B = 0;
  DevBuf<double> v64;                          // FP64 storage (precision FP64)
  DevBuf<float> v32;                           // FP32 storage (mixed precision)
  // inverses of the 64x64 diagonal blocks of the factors (row-major, identity-padded past
  // the end of a matrix), block b of matrix j at boff[j] + 4096 b; same precision as v
  std::vector<int64_t> boff;
  DevBuf<int64_t> d_boff;
  DevBuf<double> dinv64;
  DevBuf<float> dinv32;
  bool fp32 = false;
  int solve_groups[2] = {0, 0};                // work-groups per matrix: 1-RHS, m-RHS solve
  int force_groups[2] = {0, 0};                // requested (0: automatic, capped by residency)
  int share = 1;                               // contexts whose solves may run concurrently
  DevBuf<int> err;                             // error word of the solves (poll time-out)
  bool coarse = false;                         // the coarse matrix (own solve kernel name)
  // column panels of solves with more right-hand sides than one launch takes
  DevBuf<double> panel;
  DevBuf<int64_t> d_poff;
  // forward solutions of the single-right-hand-side solve (64-aligned segment per matrix)
  DevBuf<double> ybuf;
  DevBuf<int64_t> d_yoff;
  DevBuf<double> mbuf;                         // the same for up to 32 right-hand sides
};

// Addresses of one matrix in a solve over the factors of several band sets in one launch
struct BandPtrs {
  const void* v;                               // factor (precision of the launch)
  const void* dinv;                            // inverse 64x64 diagonal blocks
  double* x;                                   // right-hand side in, solution out
  double* y;                                   // forward-solution scratch (64-aligned length)
  double* z;                                   // backward-solution scratch
  int64_t n, B;                                // rows, half-bandwidth
  const int64_t* fcb;                          // envelope by 64-row blocks (see BandSet)
  const int64_t* lrb;
  int64_t G;                                   // work-groups sharing the matrix
};

// The single-right-hand-side solves of several band sets of one precision on one device in
// one launch (the subdomain solves of many independent systems advanced in lockstep)
struct MultiSolve {
  std::vector<BandSet*> sets;                  // in table order
  std::vector<BandPtrs> host;
  DevBuf<BandPtrs> tab;
  DevBuf<int32_t> work;                        // (matrix, group) per work-group, -1: none
  DevBuf<int> err;                             // time-out word of the launches
  int n_mat = 0, n_wg = 0;
  int64_t max_n = 0;
  bool fp32 = false;
};

struct Schwarz {
  int n_sub = 0, W = 0;                        // subdomains, 64-bit mask words
  DevBuf<uint64_t> elem_mask, node_or, node_and;
  // per subdomain node lists (interior I, Neumann D), concatenated, with offsets
  std::vector<int64_t> nI, nD, offI, offD, nE, offE;
  DevBuf<int64_t> d_offI, d_offD, d_nI, d_nD, d_offE, d_nE;
  DevBuf<int32_t> I_nodes, D_nodes, E_list;
  DevBuf<int32_t> I_loc, D_loc;                // [n_sub * n_nodes], -1 when absent
  DevBuf<int32_t> node_cnt;                    // subdomains holding the node as interior
  BandSet A;                                   // interior factors L_j
  DevBuf<double> dg;                           // diagonal of K (scaling of FP32 factors)
  std::vector<int64_t> xoff;                   // local vector segment of each subdomain
  DevBuf<int64_t> d_xoff;
  // coarse space
  bool two_level = false;
  std::vector<int32_t> nev;
  std::vector<int64_t> z_off;                  // offset of Z_j (row-major nI_j*3 x nev_j)
  DevBuf<int64_t> d_z_off;
  DevBuf<int32_t> d_nev, d_c_off;              // coarse column offset of each subdomain
  std::vector<int32_t> c_off;
  int64_t n0 = 0;
  DevBuf<double> Z;
  BandSet C;                                   // Cholesky factor of K_0 (full band)
  DevBuf<int64_t> d_c_xoff;
  std::vector<std::vector<double>> lam;        // eigenvalues kept per subdomain
  // work vectors for applying P
  DevBuf<double> wr64, wx64;                   // gathered local rhs / solution (FP64)
  DevBuf<double> y0, y0b;                      // coarse rhs / solution
  DevBuf<double> y0part;                       // per-subdomain partial restriction
  int precision = GX_FP64;
};

}  // namespace gx

struct gx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // mesh copy
  int64_t n_nodes = 0, n_elems = 0;
  gx::DevBuf<double> xyz;
  gx::DevBuf<int32_t> conn, elayer;
  gx::DevBuf<uint32_t> wrap;                   // periodic meshes: element nodes at the seam
  double period[3] = {0.0, 0.0, 0.0};
  gx::DevBuf<int32_t> ne_ptr, ne_idx;          // node -> element incidence (sorted)
  gx::DevBuf<uint8_t> fixed;                   // per DOF: 1 if clamped
  // element matrices, block-major: Ke[((e * 20 + a) * 20 + b) * 9 + 3 i + k]
  gx::DevBuf<double> Ke;
  // K: 3x3-block CSR
  gx::DevBuf<int32_t> row_ptr, col;
  gx::DevBuf<double> val;
  int64_t nnzb = 0;
  bool assembled = false;
  bool matrix_only = false;                    // K given by gx_matrix_load (no mesh)
  // preconditioner
  gx::Schwarz sw;
  bool setup_done = false;
  // PCG work vectors
  gx::DevBuf<double> r, z, p, q, bm, red;
  gx::HostBuf<double> hred;                    // the reduction scalars, read by the host
  int32_t pcg_iters = 0;
  int32_t eig_iters = 0;
  int64_t neumann_entries = 0;
  int64_t neumann_envelope = 0;                // envelope entries of the eigensolver's factors
  double neumann_flops = 0.0;                  // their band Cholesky flops
  int32_t fp64_fallbacks = 0;                  // bit 0: interior, bit 1: eigensolver factors
  double phase_ms[8] = {0};
  // the eigensolver's multi-right-hand-side band solves of the last setup (HIP events)
  double mrhs_ms = 0.0, mrhs_bytes = 0.0;
  int64_t mrhs_calls = 0;
  int tune[4] = {0, 0, 0, 0};                  // see gx_tune
  // contexts set up at once on the device (gx_geneo_setup_batch): the set-up's
  // multi-work-group launches take this share of the machine's resident capacity
  int share = 1;
  // materials and loads of the last assembly (kept for the sensitivities)
  int32_t n_layers = 0;
  std::vector<double> eng;                     // 9 engineering constants per layer
  gx::DevBuf<double> Cl, ang;                  // layer stiffness (material axes), ply angle
  int64_t n_faces = 0;
  gx::DevBuf<int32_t> face_e, face_id;
  gx_traction traction{};
};

namespace gx {
// implemented in the respective .hip files
void build_node_elem(gx_ctx* c);
void spmv(gx_ctx* c, const double* x, double* y);
void geneo_setup(gx_ctx* c, const gx_geneo_opts* o, int32_t* nev_out, int64_t* n0_out);
void precond_apply(gx_ctx* c, const double* r, double* z);
void dd_build(gx_ctx* c, const int32_t* part, int n_sub, int overlap);
void interior_factors(gx_ctx* c, int precision);
// after_factor (if set) runs once the eigensolver's shifted Neumann matrices are factored
void geneo_coarse(gx_ctx* c, const gx_geneo_opts* o,
                  const std::function<void()>& after_factor = nullptr);
// half bandwidths (DOFs) of K restricted to each list; env_out (optional): the envelope
// entries of each restricted matrix's lower triangle, diagonal included
std::vector<int64_t> list_bandwidth(gx_ctx* c, const int32_t* list, const int64_t* d_off,
                                    const int64_t* d_cnt, const int32_t* loc,
                                    const std::vector<int64_t>& cnt,
                                    std::vector<int64_t>* env_out = nullptr,
                                    std::vector<int32_t>* first_out = nullptr);
double interior_refactor_ms(gx_ctx* c);
// first_node (optional): for each matrix's nodes in order (n_j / 3 each, concatenated),
// the first node its rows couple to; it gives the envelope (env, env_flops, the block
// tables), otherwise the band itself is taken
void band_layout(BandSet& bs, const std::vector<int64_t>& n, const std::vector<int64_t>& B,
                 bool fp32, hipStream_t st, const std::vector<int32_t>* first_node = nullptr);
void band_factor(BandSet& bs, hipStream_t st, const char* what);
// A banded factorisation in flight (band_factor_start enqueues it on st, band_factor_finish
// waits for it and raises GX_ENOTSPD on a non-positive pivot).  It owns the look-ahead
// stream, the diagonal-block scratch and the pivot-error word; its destructor waits for
// both streams first, so none of them is released while a kernel of the job may run.
struct FactorJob {
  hipStream_t st = nullptr;
  std::string what;
  DevBuf<int> err;
  DevBuf<double> inv;                          // inverse diagonal blocks handed over
  DevBuf<int> flags;                           // per panel block: epoch of its completion;
                                               // then per launch: the work-group counter
  hipStream_t la = nullptr;                    // trailing-update stream (default priority)
  hipEvent_t chain = nullptr, rest[2] = {nullptr, nullptr};
  std::thread launcher;                        // enqueues the launches of a threaded job
  std::exception_ptr launch_error;
  FactorJob() = default;
  ~FactorJob();
  FactorJob(const FactorJob&) = delete;
  FactorJob& operator=(const FactorJob&) = delete;
};
// threaded: a host thread of the job enqueues the launches, so the caller goes on at once
// (a long chain of launches blocks the enqueuing thread once the device's queues are
// full); band_factor_finish joins it.
void band_factor_start(BandSet& bs, hipStream_t st, FactorJob& job, const char* what,
                       bool threaded = false);
void band_factor_finish(FactorJob& job);
// The interior factorisation as a job that can run on a side stream (see schwarz.hip).
struct InteriorJob {
  std::vector<int64_t> n, B, env;
  std::vector<int32_t> first;                  // first coupled node of every node
  int64_t maxI = 0;
  bool fp32 = false;
  FactorJob factor;
};
void interior_factors_start(gx_ctx* c, int precision, hipStream_t s, InteriorJob& job);
// the same in two parts: the bandwidths, layout, allocation and band fill (enqueued on s),
// then the factorisation's launches
void interior_factors_prepare(gx_ctx* c, int precision, hipStream_t s, InteriorJob& job);
void interior_factors_launch(gx_ctx* c, hipStream_t s, InteriorJob& job, bool threaded);
void interior_factors_finish(gx_ctx* c, InteriorJob& job);
void band_solve_check(BandSet& bs, hipStream_t st);
void band_solve(BandSet& bs, const int64_t* d_xoff, double* x, hipStream_t st, int ncol = 1,
                const int32_t* active = nullptr);
// Algorithmic bytes of one forward-and-backward solve with ncol right-hand sides: the
// factor's envelope read once per sweep (2 w sum env_j) plus the FP64 right-hand side and
// solution passes (32 n_j ncol); band = true counts the stored band and the inverse diagonal
// blocks that the kernels read instead of the envelope.
double band_solve_bytes(const BandSet& bs, int ncol, const int32_t* active_host = nullptr,
                        bool band = false);
void multi_solve_plan(MultiSolve& m, const std::vector<BandSet*>& sets,
                      const std::vector<double*>& x, const std::vector<const int64_t*>& xoff,
                      hipStream_t st);
void multi_solve(MultiSolve& m, hipStream_t st);
void multi_solve_check(MultiSolve& m, hipStream_t st);
void precond_local(gx_ctx* c, const double* r);
void precond_finish(gx_ctx* c, const double* r, double* z);
void laminate_velocity(const gx_laminate* lam, int param, double* xd, hipStream_t st);
void laminate_region(const gx_laminate* lam, uint8_t* mask, hipStream_t st);
void laminate_sizes(const gx_laminate* lam, int64_t* n_nodes, int64_t* n_elems);
// device address of the allocation-free entry points' scratch array (adjoint.hip), resolved
// once per device with that device current
void noalloc_scratch_init(int device);
// HIP event pair on a stream (timing of single launches)
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    GX_HIP(hipEventCreate(&a));
    GX_HIP(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  float ms() const {
    float t = 0;
    GX_HIP(hipEventSynchronize(b));
    GX_HIP(hipEventElapsedTime(&t, a, b));
    return t;
  }
};

struct Timer {
  hipStream_t s;
  std::chrono::steady_clock::time_point t0;
  explicit Timer(hipStream_t st) : s(st) {
    (void)hipStreamSynchronize(s);
    t0 = std::chrono::steady_clock::now();
  }
  double ms() {
    (void)hipStreamSynchronize(s);
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
        .count();
  }
};
}  // namespace gx

#define GX_API_BEGIN(ctx)                                                             \
  if (!(ctx)) return GX_EINVAL;                                                       \
  try {                                                                               \
    ::gx::CtxScope gx_scope_(ctx);                                                    \
    (ctx)->err.clear();                                                               \
    GX_HIP(hipSetDevice((ctx)->device));

#define GX_API_END(ctx)                                                               \
  }                                                                                   \
  catch (const ::gx::Error& e_) {                                                     \
    (ctx)->err = e_.what();                                                           \
    return e_.code;                                                                   \
  }                                                                                   \
  catch (const std::exception& e_) {                                                  \
    (ctx)->err = e_.what();                                                           \
    return GX_EINVAL;                                                                 \
  }                                                                                   \
  return GX_OK;
