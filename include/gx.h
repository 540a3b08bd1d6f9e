/*
 * gx — AS-GenEO preconditioned conjugate gradients for laminated composites on one
 * AMD Instinct MI355X (gfx950).
 *
 * The library solves the linear elasticity system K u = f of the paper's Eq. (eq-1)
 * (Reinarz et al., "dune-composites", section 2.3) for layered composites meshed with
 * 20-node serendipity hexahedra (section 2.1), by CG on P K u = P f (Eq. eq-pre) with P
 * the two-level overlapping additive Schwarz preconditioner whose coarse space is built
 * from local generalised eigenproblems (GenEO, section 2.3).
 *
 * Conventions (all entry points)
 *   - Units: mm, N, MPa.  Indices are 0-based.
 *   - A displacement-sized vector has 3 * n_nodes FP64 entries, DOF = 3 * node + component
 *     (x, y, z).  Clamped DOFs carry 0 on output; their input values are ignored.
 *   - Arrays whose length grows with the mesh are DEVICE pointers (e.g. a torch tensor's
 *     data_ptr() on the context's device); descriptor structs and per-layer / per-subdomain
 *     tables are HOST pointers.  Every input is borrowed for the duration of the call only:
 *     the library copies what it keeps.
 *   - All work is queued on the context's HIP stream; calls return after that work has
 *     completed (results are ready for any stream).
 *   - No exception crosses this interface.  Every call returns a gx_status; on failure a
 *     message is available from gx_last_error().
 *   - A context is used by one host thread at a time; different contexts may be used from
 *     different threads at once (the library's shared state, a cache of released device
 *     blocks, is locked).
 *   - Library-owned state (mesh copy, element matrices, K, decomposition, factors, coarse
 *     space) lives in the context and is released by gx_destroy().
 */
#ifndef GX_H
#define GX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gx_ctx gx_ctx;
typedef int32_t gx_status;

enum {
  GX_OK = 0,
  GX_EINVAL = 1,      /* bad argument (null pointer, size, unsupported option) */
  GX_ENOMEM = 2,      /* device allocation failed */
  GX_EHIP = 3,        /* a HIP runtime call failed */
  GX_ENOTSPD = 4,     /* non-positive pivot in a Cholesky factorisation */
  GX_ENOCONV = 5,     /* iteration limit reached; outputs hold the last iterate */
  GX_EBREAKDOWN = 6,  /* CG breakdown: p^T K p <= 0 or not finite */
  GX_ESTATE = 7       /* call made out of order (e.g. solve before setup) */
};

enum { GX_GEOM_FLAT = 0, GX_GEOM_LSECTION = 1 };
enum { GX_FP64 = 0, GX_MIXED = 1 };

/* ------------------------------------------------------------------------------------
 * Context
 * ------------------------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to queue work on,
 * or NULL to let the library create (and own) one. */
gx_status gx_create(gx_ctx** ctx, int32_t device, void* hip_stream);
void gx_destroy(gx_ctx* ctx);
/* Message of the last failed call on this context ("" if none).  Never NULL. */
const char* gx_last_error(const gx_ctx* ctx);
/* Library version string. */
const char* gx_version(void);

/* ------------------------------------------------------------------------------------
 * Laminate mesh (sections 2.2 and 3: tensor-product laminate grids; the flat ->
 * wrinkled -> curved mapping of Eq. eq-wrinkle and the curved map that follows it).
 *
 * Layers are listed from zeta = 0 (inner radius / bottom) outwards, each split into
 * layer_nel equal element layers.  Along s the flat part has nx equal elements over
 * `length`; the L-section has nx_limb equal elements on each straight limb of length
 * `limb` and nx - 2 nx_limb equal elements on a 90 degree arc of mid-surface radius
 * radius + T/2 centred at (limb, 0) (T = total thickness), s = 0 at mid-arc.  Along l
 * there are ny equal elements over `width`.  The wrinkle displaces every layer by
 * w(s - s_c) = A exp(-((s - s_c)/L)^2) cos(2 pi (s - s_c)/L) along the laminate normal
 * (s_c = length/2 for a flat part, 0 for the L-section); A = 0 disables it.
 *
 * Node numbering: nodes sit on a doubled lattice (i2, j2, k2) with at most one odd index
 * (8 vertices and 12 edge midpoints per element, section 2.1); the node number is the rank
 * of (k2, j2, i2) in lexicographic order, i2 fastest.  Element e = (ez * ny + ey) * nx + ex.
 * Element-local node order: 8 vertices (di, dj, dk) lexicographic with di fastest; then
 * x-directed edges at (dj, dk) = (0,0),(1,0),(0,1),(1,1); y-directed at (di, dk); z-directed
 * at (di, dj).
 * ------------------------------------------------------------------------------------ */
typedef struct {
  int32_t geometry;          /* GX_GEOM_FLAT or GX_GEOM_LSECTION */
  int32_t nx, ny;            /* elements along s and along l */
  int32_t nx_limb;           /* L-section only: elements on each limb */
  int32_t n_layers;          /* material layers (<= 96) */
  const double* layer_t;     /* host [n_layers] thickness (mm) */
  const int32_t* layer_nel;  /* host [n_layers] element layers (>= 1) */
  double length;             /* flat only: extent along s (mm) */
  double width;              /* extent along l (mm) */
  double radius, limb;       /* L-section only: inner radius and limb length (mm) */
  double wrinkle_amp, wrinkle_len;  /* A and L of w(s) (mm) */
  /* The paper's localised wrinkle defect (section 3, Eq. eq-f), L-section only, added to
   * the shift w(s): f = d sech^2(s_p / b1) sech^2(pi (zeta - zeta_def) / (R b2))
   * sech^2(pi (l - l_def) / (W b3)), s_p = 2 (s - s_def) / (R + T/2) (the paper's arc
   * parameter, 0..pi over the 90 degree arc), b2 = b2_in below zeta_def and b2_out above,
   * R the inner radius.  defect_amp = 0 disables it. */
  double defect_amp;                         /* d (mm) */
  double defect_s, defect_l, defect_zeta;    /* centre: arc length from mid-arc, position
                                                across the width, height above the inner
                                                surface (mm) */
  double defect_b1, defect_b2_in, defect_b2_out, defect_b3;
  /* Graded meshes (section 2.2: bias ratios 400 across the width and 10 through each layer;
   * section 3.1: 2 towards the defect): the ratio of the largest to the smallest element,
   * sizes growing geometrically and symmetric about the segment's middle; <= 1: uniform.
   * bias_s: a flat part towards mid-length, the arc of an L-section towards mid-arc (limbs
   * uniform); bias_l: across the width towards the laminate's edges; bias_z: every layer
   * towards its two faces. */
  double bias_s, bias_l, bias_z;
  /* Resin edge strips (sections 2.2 and 3): strips of strip_width (mm, 0: none) at l = 0
   * and l = width with strip_ny uniform elements each (the laminate between them takes the
   * other ny - 2 strip_ny elements); their elements take ply-stack entry strip_mat. */
  double strip_width;
  int32_t strip_ny, strip_mat;
  /* The stiff end layer carrying the moment (section 2.2): end_column = 1 gives the last
   * element column along s ply-stack entry end_mat. */
  int32_t end_column, end_mat;
  /* Periodic boundary conditions across the width (section 3: a very wide part; section
   * 2.1): periodic_l = 1 identifies the nodes at l = width with those at l = 0 (they are
   * not separate nodes).  The elements of the last column then reach across the seam: their
   * nodes there take the coordinates of the l = 0 nodes plus the width along l, which
   * gx_laminate_wrap describes for gx_assemble.  Not with edge strips. */
  int32_t periodic_l;
} gx_laminate;

/* Node, element, clamped-node and loaded-face counts of a laminate (host only). */
gx_status gx_laminate_counts(const gx_laminate* lam, int64_t* n_nodes, int64_t* n_elems,
                             int64_t* n_clamped, int64_t* n_faces);

/* Build the mesh on the device: xyz [3 n_nodes], conn [20 n_elems], elem_layer [n_elems]
 * (material layer index of each element), all device buffers sized by gx_laminate_counts.
 * Also fills the boundary lists: clamped [n_clamped] (every node on the s = s_min end,
 * all three components fixed, section 2.2) and the loaded faces face_elem/face_id
 * [n_faces] (local face 1 = xi = +1 of the elements on the s = s_max end).
 * Any of the boundary pointers may be NULL. */
gx_status gx_laminate_mesh(gx_ctx* ctx, const gx_laminate* lam, double* xyz, int32_t* conn,
                           int32_t* elem_layer, int32_t* clamped, int32_t* face_elem,
                           int32_t* face_id);

/* Which element nodes of a periodic laminate stand for its seam (device [n_elems]): bit a of
 * elem_wrap[e] is set when node a of element e is a node at l = 0 that the element uses at
 * l = width (its coordinates plus the period); zero for a laminate that is not periodic. */
gx_status gx_laminate_wrap(gx_ctx* ctx, const gx_laminate* lam, uint32_t* elem_wrap);

/* Box partition of a laminate into px * py in-plane subdomains of element index ranges
 * (full thickness), box p along an axis of n elements covering [p n / P, (p + 1) n / P)
 * (section 2.3: subdomains of roughly equal size).  elem_part: device [n_elems], value
 * iy * px + ix. */
gx_status gx_laminate_partition(gx_ctx* ctx, const gx_laminate* lam, int32_t px, int32_t py,
                                int32_t* elem_part);

/* Parameters of the end load of a laminate (host only):
 * kind 0: uniform traction `value[0..2]` (MPa);
 * kind 1: end moment value[0] per unit width (N mm / mm), applied as the linear normal
 *         traction -12 M (zeta - T/2) / T^3 on the s = s_max face, which has zero force
 *         resultant and puts the inner face in tension along the limb (opens a corner,
 *         section 2.2). */
typedef struct {
  double t0[3];     /* uniform traction vector (MPa) */
  double k;         /* linear normal part: t += k * ((x - c) . d) * n_out */
  double c[3], d[3];
} gx_traction;
gx_status gx_laminate_traction(const gx_laminate* lam, int32_t kind, const double* value,
                               gx_traction* out);

/* ------------------------------------------------------------------------------------
 * Assembly of K and f (Eq. eq-1; section 2.1: full 3x3x3 Gauss integration).
 * ------------------------------------------------------------------------------------ */
typedef struct {
  int32_t n_layers;
  const double* eng;        /* host [9 n_layers]: E1 E2 E3 G12 G13 G23 nu12 nu13 nu23 (MPa)
                               of each material layer in its material axes (Table 1);
                               G12 <= 0 marks an isotropic layer given by E = E1 and
                               nu = nu12 alone (shear modulus E / (2 (1 + nu))) */
  const double* angle_deg;  /* host [n_layers]: ply angle, fibre = cos(a) e1 + sin(a) e2
                               about the local normal e3 (e1 along s, e2 along l) */
} gx_plystack;

typedef struct {
  int64_t n_nodes, n_elems;
  const double* xyz;        /* device [3 n_nodes] */
  const int32_t* conn;      /* device [20 n_elems], element-local order above */
  const int32_t* elem_layer;/* device [n_elems], index into the ply stack */
  /* periodic meshes (or NULL): device [n_elems]; element e sees node a at its coordinates
   * plus period[] when bit a of elem_wrap[e] is set (e.g. from gx_laminate_wrap) */
  const uint32_t* elem_wrap;
  double period[3];
} gx_mesh;

typedef struct {
  int64_t n_clamped;
  const int32_t* clamped;   /* device [n_clamped] nodes with all three components fixed */
  int64_t n_faces;
  const int32_t* face_elem; /* device [n_faces] */
  const int32_t* face_id;   /* device [n_faces] local face: 0/1 = xi -/+, 2/3 eta, 4/5 zeta */
  gx_traction traction;
} gx_loads;

/* Assemble the stiffness K (kept in the context as 3x3-block CSR over all nodes, clamped
 * DOFs replaced by identity rows and columns) and the load vector f_out (device
 * [3 n_nodes], zero on clamped DOFs).  The material stiffness is rotated at every Gauss
 * point into the frame e1 = unit dx/dxi, e2 = unit part of dx/deta orthogonal to e1,
 * e3 = e1 x e2, then by the ply angle about e3.  Any previous setup is discarded. */
gx_status gx_assemble(gx_ctx* ctx, const gx_mesh* mesh, const gx_plystack* plies,
                      const gx_loads* loads, double* f_out);

/* Number of block rows (= nodes) and 3x3 blocks of K. */
gx_status gx_matrix_info(gx_ctx* ctx, int64_t* n_block_rows, int64_t* n_blocks);
/* Copy K out: row_ptr device [n_block_rows + 1], col device [n_blocks], val device
 * [9 n_blocks] (each block row-major).  Columns are sorted within each row. */
gx_status gx_matrix_copy(gx_ctx* ctx, int32_t* row_ptr, int32_t* col, double* val);
/* Install a 3x3-block matrix given by the caller as K (in place of gx_assemble), for
 * gx_spmv, gx_matrix_info and gx_matrix_copy: n_block_rows block rows, n_blocks blocks,
 * row_ptr [n_block_rows + 1], col [n_blocks], val [9 n_blocks] (each block row-major),
 * host or device pointers, copied.  Rows may be empty, columns need not be sorted.  The
 * mesh-dependent calls (set-up, objective, adjoint, failure criterion) then return
 * GX_ESTATE.  GX_EINVAL for inconsistent row pointers or out-of-range columns. */
gx_status gx_matrix_load(gx_ctx* ctx, int64_t n_block_rows, int64_t n_blocks,
                         const int32_t* row_ptr, const int32_t* col, const double* val);
/* y = K x (device vectors of 3 n_nodes). */
gx_status gx_spmv(gx_ctx* ctx, const double* x, double* y);

/* ------------------------------------------------------------------------------------
 * Two-level overlapping Schwarz preconditioner with GenEO coarse space (section 2.3).
 * Subdomain j grows its core elements `overlap` times by every element sharing a node;
 * its local problem is K restricted to the DOFs of nodes all of whose elements lie in the
 * subdomain (zero displacement on the artificial boundary), solved exactly by a banded
 * Cholesky factorisation.  The partition of unity is 1 / (number of subdomains holding a
 * DOF as interior).  GenEO: A_j^N p = lambda X_j A_j^o X_j p on the DOFs of the
 * subdomain's nodes (A^N over the subdomain's elements, A^o over those also in another
 * subdomain); the coarse vectors are the partition of unity times the eigenvectors with
 * lambda < tau (at most nev_max), or the nev smallest when nev > 0.
 * ------------------------------------------------------------------------------------ */
typedef struct {
  int32_t n_sub;
  const int32_t* elem_part;  /* device [n_elems]: core subdomain of each element */
  int32_t overlap;           /* element layers of overlap (>= 1) */
  double tau;                /* eigenvalue threshold (used when nev <= 0) */
  int32_t nev;               /* > 0: fixed number of modes per subdomain (<= 40) */
  int32_t nev_max;           /* cap per subdomain (<= 32) */
  int32_t precision;         /* GX_FP64, or GX_MIXED: FP32 subdomain factors and solves */
  int32_t coarse;            /* 1: two-level (GenEO); 0: one-level Schwarz */
  const int32_t* nev_per_sub;/* optional host [n_sub]: modes per subdomain (overrides) */
  double eig_tol;            /* eigenpair backward-error target ||M x - theta B x|| <=
                                eig_tol S ||x||, S = max over the block of ||M x|| / ||x||
                                (0: default 1e-4) */
  int32_t eig_maxit;         /* eigensolver iteration cap (0: default 1000) */
} gx_geneo_opts;

/* Build the decomposition, factor the subdomain matrices, solve the local eigenproblems
 * and factor the coarse matrix K_0 = Z^T K Z.  nev_out: host [n_sub] modes kept per
 * subdomain (may be NULL); n0_out: coarse dimension (may be NULL). */
gx_status gx_geneo_setup(gx_ctx* ctx, const gx_geneo_opts* opts, int32_t* nev_out,
                         int64_t* n0_out);

/* Set-up of many contexts (extension: many laminates at once): gx_geneo_setup(ctxs[i],
 * opts[i], nev_out[i], n0_out + i) for every i, up to `concurrent` of them at a time on
 * host threads of the library, each context on its own stream.  While they run, each
 * context's multi-work-group launches take 3/4 of the device's resident capacity divided
 * by min(concurrent, n), so that concurrent launches stay resident together.  Set-ups are
 * chains of small launches on a few streams each, so they overlap only as far as the
 * process has hardware queues (GPU_MAX_HW_QUEUES, read when the HIP runtime starts;
 * HIP's default is 4).  Each
 * context appears once and its stream is not used by the caller meanwhile.  nev_out
 * (host array of n host pointers, each NULL or [opts[i]->n_sub]), n0_out and status_out
 * (host [n]) may be NULL.  Returns GX_EINVAL for bad arguments (nothing run), else GX_OK
 * if every set-up succeeded, else the first non-OK status (each context's gx_last_error
 * explains its own). */
gx_status gx_geneo_setup_batch(int32_t n, gx_ctx* const* ctxs, const gx_geneo_opts* const* opts,
                               int32_t concurrent, int32_t* const* nev_out, int64_t* n0_out,
                               int32_t* status_out);

/* Per-subdomain sizes: interior DOFs, Neumann DOFs, half bandwidth of the interior factor
 * (host arrays [n_sub], any may be NULL). */
gx_status gx_subdomain_info(gx_ctx* ctx, int64_t* n_interior, int64_t* n_neumann,
                            int64_t* half_band);
/* GenEO eigenvalues of subdomain j: lam host [nev_out[j]]. */
gx_status gx_geneo_eigenvalues(gx_ctx* ctx, int32_t j, double* lam);

/* z = P r (device vectors of 3 n_nodes). */
gx_status gx_precond_apply(gx_ctx* ctx, const double* r, double* z);

/* ------------------------------------------------------------------------------------
 * Preconditioned CG (section 2.3): x (device, in: initial guess, out: solution) for
 * K x = b; stops when ||b - K x||_2 <= rtol ||b||_2 (recurrence residual), or after maxit
 * iterations (GX_ENOCONV, x holds the last iterate).  iters_out: CG iterations (products
 * with K inside the loop); relres_out: final ||r|| / ||b||; hist: host [maxit + 1] or
 * NULL, relative residual before each iteration and after the last.
 * ------------------------------------------------------------------------------------ */
gx_status gx_pcg_solve(gx_ctx* ctx, const double* b, double* x, double rtol, int32_t maxit,
                       int32_t* iters_out, double* relres_out, double* hist);

/* ------------------------------------------------------------------------------------
 * Sensitivities (extension).  Objective J(u, p) = sum over the region's elements and
 * Gauss points of sigma_33^2 det J w, sigma_33 the normal stress along the laminate normal
 * of the local frame (the through-thickness stress that drives corner unfolding,
 * section 3).  region 0: every element; 1: the arc of an L-section (elements whose
 * s-range centre lies in the arc; every element of a flat laminate).  lam must be the
 * laminate whose mesh was assembled.
 * ------------------------------------------------------------------------------------ */
/* J for the displacement u (device, 3 n_nodes). */
gx_status gx_objective(gx_ctx* ctx, const gx_laminate* lam, int32_t region, const double* u,
                       double* J_out);
/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving or optimisation loops, harnesses that forbid hipMalloc): gx_objective with no
 * allocation.  Its scratch (the element mask, J per element and their sum) lives in one
 * static device array of GX_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from
 * the first gx_create on that GPU until the process ends.  The mesh must satisfy
 * 9 n_elems + 256 <= GX_NOALLOC_SCRATCH_BYTES (about 1.86 million elements), else
 * GX_EINVAL and nothing is launched.  Every call on a GPU shares that GPU's array and
 * overwrites what the last call left there (nothing in it needs to start at zero), so
 * calls that overlap in time on one GPU, from any contexts or threads, race.  J equals
 * gx_objective's bit for bit (same kernels, same summation order). */
#define GX_NOALLOC_SCRATCH_BYTES (16u << 20)
gx_status gx_objective_noalloc(gx_ctx* ctx, const gx_laminate* lam, int32_t region,
                               const double* u, double* J_out);
/* J and dJ/dp by the adjoint method: K lambda = dJ/du is solved by PCG with the current
 * preconditioner to rtol (iters_out: its iterations), then
 * dJ/dp = dJ/dp|_u - lambda^T (dK/dp u - df/dp).  dJdp (host) receives 2 + n values, n the
 * entries of the assembled ply stack (the laminate's layers, then any extra materials such
 * as edge strips): [0] wrinkle amplitude, [1] wrinkle wavelength, [2 + k] the modulus E11
 * of entry k (E for an isotropic one), in the units of J per mm and per MPa.  u must solve the
 * assembled system (e.g. gx_pcg_solve to a tight tolerance).  GX_ENOCONV if the adjoint
 * solve does not reach rtol in maxit iterations (the outputs are still filled, from its
 * last iterate); GX_ESTATE before gx_geneo_setup. */
gx_status gx_adjoint(gx_ctx* ctx, const gx_laminate* lam, int32_t region, const double* u,
                     double rtol, int32_t maxit, double* J_out, double* dJdp,
                     int32_t* iters_out);

/* ------------------------------------------------------------------------------------
 * Delamination onset (section 3.3, Eq. eq-Camanho): at the 27 Gauss points of every
 * element of the selected layers the stresses of u are recovered in the local frame
 * (s, l, r) = (e1, e2, e3) of the assembly (the strain rotated into the material axes, times
 * the layer stiffness, turned back by the ply angle), and
 *   F = sqrt((max(sigma_r, 0) / s33)^2 + (tau_rs / s13)^2 + (tau_rl / s13)^2).
 * The paper applies it in the resin interface layers with s33 = 61 MPa, s13 = 97 MPa;
 * failure initiates at F = 1, i.e. at the load scaled by 1 / F_max (linear problem).
 * layer_mask: host [n_layers of the ply stack], nonzero = evaluate the layer; NULL selects
 * the isotropic entries.  F_gauss (device [27 n_elems], point q = 9 k + 3 j + i with i along
 * xi) and F_elem (device [n_elems], the element's maximum) may be NULL; both are 0 outside
 * the selected layers.  out (host) receives the maximum, where it occurs (ties: the lowest
 * element, then the lowest point) and the local stresses there, in MPa, ordered
 * sigma_s, sigma_l, sigma_r, tau_lr, tau_sr, tau_sl.  Deterministic.
 * ------------------------------------------------------------------------------------ */
typedef struct {
  double F_max;
  int64_t elem;
  int32_t gauss;
  int32_t layer;            /* ply-stack entry of that element */
  double stress[6];
} gx_failure_result;
gx_status gx_failure(gx_ctx* ctx, const double* u, const int32_t* layer_mask, double s33,
                     double s13, double* F_gauss, double* F_elem, gx_failure_result* out);

/* The subdomain solver on its own: batched banded Cholesky factorisation and triangular
 * solves (section 2.4: the local problems are solved exactly by a direct method).
 * n_mat matrices; matrix j has order n[j] and half bandwidth bw[j] (host arrays) and is
 * given in row-major band storage: entry (r, c), r - bw[j] <= c <= r, at
 * off_j + r (bw[j] + 1) + (c - r + bw[j]), off_j = sum over i < j of n[i] (bw[i] + 1)
 * (device, FP64; copied, the input is not modified).  x (device) holds nrhs right-hand
 * sides per matrix, row-major n[j] x nrhs, matrices concatenated; overwritten with the
 * solutions.  nrhs is 1 or a multiple of 8 up to 64 (more than 32 are solved in panels of
 * 32).  precision GX_MIXED factors and solves with FP32 factors of
 * diag(A)^-1/2 A diag(A)^-1/2 (x stays FP64).  groups > 0 forces the number of
 * work-groups per matrix (bounded by what stays resident), 0 chooses it.  GX_ENOTSPD on a
 * non-positive pivot. */
gx_status gx_band_factor_solve(gx_ctx* ctx, int32_t n_mat, const int64_t* n, const int64_t* bw,
                               const double* band, int32_t precision, int32_t nrhs,
                               int32_t groups, double* x);

/* Batched PCG (extension: many laminates at once).  n contexts, each set up
 * (gx_geneo_setup) for its own laminate and, for overlap, on its own HIP stream, solve
 * K_i x_i = b_i in lockstep: every iteration enqueues the work of each unconverged system on
 * its stream, the subdomain solves of all of them as one launch per device and factor
 * precision (on a stream of the batch's own that waits for the systems' streams and that
 * they wait for), and then waits once for all of them; a system leaves the batch when it
 * converges (the stopping test of gx_pcg_solve, per system).  Each context appears once
 * (GX_EINVAL otherwise).  b[i], x[i]: device vectors of context i (x[i] in: initial
 * guess).  iters_out, relres_out, status_out: host [n] (may be NULL).  Returns GX_OK if
 * every system converged, else the first non-OK status (each context's gx_last_error
 * explains its own). */
gx_status gx_pcg_solve_batch(int32_t n, gx_ctx* const* ctxs, const double* const* b,
                             double* const* x, double rtol, int32_t maxit, int32_t* iters_out,
                             double* relres_out, int32_t* status_out);

/* Measurement of one library kernel with HIP events on the context's stream: the average
 * duration over `reps` launches (ms) and the algorithmic bytes one launch must move
 * (bytes, 0 when not defined).  which: 0 = block-CSR product y = K x; 1 = the batched
 * subdomain band solves of one preconditioner application (forward and backward);
 * 2 = one whole preconditioner application; 3 = the coarse solve; 4 = the GenEO
 * eigensolver's multi-right-hand-side band solves, as timed during the last
 * gx_geneo_setup (average per solve; reps is ignored); 5 = the Cholesky factorisation of
 * the subdomain matrices (section 2.4), refilled from K and factored again alone on the
 * stream (the factors come out unchanged) - `bytes` then receives its flops instead (the
 * Cholesky count over the envelope, sum over columns of h^2 + 2 h + 1 with h the rows
 * below the diagonal inside the envelope).  The algorithmic bytes of a band solve are the factor's envelope
 * (profile: every row from its first nonzero column to the diagonal, where Cholesky
 * creates all its fill) read once per sweep, 2 w sum_j env_j with w = 8 (FP64) or 4
 * (FP32 factors), plus four FP64 passes over the right-hand sides (32 n_j per column). */
gx_status gx_kernel_time(gx_ctx* ctx, int32_t which, int32_t reps, double* avg_ms,
                         double* bytes);

/* Tuning knobs, applied by the next gx_geneo_setup (0 = automatic choice):
 * param 0: work-groups per subdomain for the single right-hand-side band solves (PCG);
 * param 1: work-groups per subdomain for the multi-column band solves (eigensolver).
 * Values 1..8; the library lowers a request that would not keep every work-group of the
 * pipelined launch resident on the device.  The batched PCG (gx_pcg_solve_batch) plans the
 * work-groups of its joint subdomain solve itself and ignores param 0. */
gx_status gx_tune(gx_ctx* ctx, int32_t param, int64_t value);

/* Counters of the last setup / solve (host [5]): eigensolver iterations, PCG iterations,
 * stored entries of the interior band factors, stored entries of the eigensolver's
 * Neumann band factors, and FP64 fall-backs of the mixed path (bit 0: an FP32 interior
 * factor broke down and the interior factors were rebuilt in FP64; bit 1: the same for the
 * eigensolver's factors). */
gx_status gx_stats(gx_ctx* ctx, int64_t* out);

/* Sizes of the subdomain factorisations of the last gx_geneo_setup (host [8]): [0] stored
 * band entries of the subdomain factors, [1] their envelope (profile) entries, [2] their
 * Cholesky flops over the envelope (column c: h^2 + 2 h + 1, h the rows below c inside the
 * envelope); [3] stored band entries of the eigensolver's Neumann factors, [4] their
 * envelope entries, [5] their flops; [6] algorithmic bytes of one PCG subdomain solve
 * (envelope, as gx_kernel_time 1 reports), [7] the bytes of the stored band, the inverse
 * diagonal blocks and the vector passes.  GX_ESTATE before gx_geneo_setup. */
gx_status gx_band_stats(gx_ctx* ctx, double* out);

/* Time spent in the last call of each phase, milliseconds (host [8], may be NULL):
 * assemble, decomposition, local factors, eigensolves, coarse, pcg, precond total in pcg,
 * spmv total in pcg. */
gx_status gx_phase_times(gx_ctx* ctx, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* GX_H */
