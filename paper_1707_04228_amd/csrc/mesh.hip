// Laminate meshes of 20-node serendipity hexahedra built on the device.
//
// Tensor-product laminate grid with a fixed number of element layers per ply and per
// interface (section 2.2), mapped flat -> wrinkled -> curved (section 3, Eq. eq-wrinkle
// and the curved map that follows it).  Every node is evaluated on the exact geometry map
// at its lattice parameter, so element edges are curved isoparametric quadratics.
#include <cmath>

#include "gx_internal.h"

namespace gx {

constexpr int MAX_LAYERS = 96;              // keeps the kernel argument block small

struct LamDev {
  int geometry, nx, ny, nz, nx_limb, n_layers;
  double length, width, radius, limb, amp, wlen, T;
  double s_a, s_b, r_ref;                        // L-section arc ends and mid radius
  double dd, ds, dl, dz, b1, b2i, b2o, b3;       // sech^2 defect (Eq. eq-f), dd = 0: none
  double bs, bl, bz;                             // bias ratios (<= 1: uniform)
  double strip_w;                                // resin edge strips (0: none)
  int strip_ny, strip_mat, end_column, end_mat;
  int periodic;                                  // lattice plane j2 = 2 ny is j2 = 0
  double t[MAX_LAYERS], z0[MAX_LAYERS];          // thickness, start of each layer
  int nel[MAX_LAYERS], cum[MAX_LAYERS + 1];      // element layers, cumulative count
};

static void check_lam(const gx_laminate* L) {
  GX_REQUIRE(L, "null laminate");
  GX_REQUIRE(L->geometry == GX_GEOM_FLAT || L->geometry == GX_GEOM_LSECTION, "geometry");
  GX_REQUIRE(L->nx >= 1 && L->ny >= 1, "nx, ny must be >= 1");
  GX_REQUIRE(L->n_layers >= 1 && L->n_layers <= MAX_LAYERS, "n_layers out of range");
  GX_REQUIRE(L->layer_t && L->layer_nel, "layer tables missing");
  for (int i = 0; i < L->n_layers; ++i)
    GX_REQUIRE(L->layer_nel[i] >= 1 && L->layer_t[i] > 0, "bad layer entry");
  GX_REQUIRE(L->width > 0, "width must be > 0");
  if (L->geometry == GX_GEOM_FLAT) GX_REQUIRE(L->length > 0, "length must be > 0");
  if (L->geometry == GX_GEOM_LSECTION) {
    GX_REQUIRE(L->radius > 0 && L->limb > 0, "radius, limb must be > 0");
    GX_REQUIRE(L->nx_limb >= 1 && L->nx - 2 * L->nx_limb >= 1, "nx_limb out of range");
  }
  if (L->wrinkle_amp != 0.0) GX_REQUIRE(L->wrinkle_len > 0, "wrinkle length must be > 0");
  GX_REQUIRE(std::isfinite(L->bias_s) && std::isfinite(L->bias_l) && std::isfinite(L->bias_z),
             "bias ratios must be finite");
  if (L->strip_width > 0) {
    GX_REQUIRE(L->strip_ny >= 1 && 2 * L->strip_ny < L->ny, "strip_ny out of range");
    GX_REQUIRE(2 * L->strip_width < L->width, "edge strips wider than the part");
    GX_REQUIRE(L->strip_mat >= 0, "strip material index");
  }
  if (L->end_column) GX_REQUIRE(L->end_mat >= 0, "end-column material index");
  if (L->periodic_l)
    GX_REQUIRE(!(L->strip_width > 0), "a periodic laminate has no free edges for strips");
  if (L->defect_amp != 0.0) {
    GX_REQUIRE(L->geometry == GX_GEOM_LSECTION, "the sech^2 defect needs an L-section");
    GX_REQUIRE(L->defect_b1 > 0 && L->defect_b2_in > 0 && L->defect_b2_out > 0 &&
                   L->defect_b3 > 0, "defect extents must be > 0");
  }
}

static LamDev make_lam(const gx_laminate* L) {
  check_lam(L);
  LamDev d;
  std::memset(&d, 0, sizeof(d));
  d.geometry = L->geometry;
  d.nx = L->nx;
  d.ny = L->ny;
  d.nx_limb = L->nx_limb;
  d.n_layers = L->n_layers;
  d.length = L->length;
  d.width = L->width;
  d.radius = L->radius;
  d.limb = L->limb;
  d.amp = L->wrinkle_amp;
  d.wlen = L->wrinkle_len > 0 ? L->wrinkle_len : 1.0;
  d.dd = L->defect_amp;
  d.ds = L->defect_s;
  d.dl = L->defect_l;
  d.dz = L->defect_zeta;
  d.b1 = L->defect_b1 > 0 ? L->defect_b1 : 1.0;
  d.b2i = L->defect_b2_in > 0 ? L->defect_b2_in : 1.0;
  d.b2o = L->defect_b2_out > 0 ? L->defect_b2_out : 1.0;
  d.b3 = L->defect_b3 > 0 ? L->defect_b3 : 1.0;
  d.bs = L->bias_s;
  d.bl = L->bias_l;
  d.bz = L->bias_z;
  d.strip_w = L->strip_width > 0 ? L->strip_width : 0.0;
  d.strip_ny = d.strip_w > 0 ? L->strip_ny : 0;
  d.strip_mat = L->strip_mat;
  d.end_column = L->end_column ? 1 : 0;
  d.end_mat = L->end_mat;
  d.periodic = L->periodic_l ? 1 : 0;
  double z = 0;
  int c = 0;
  d.cum[0] = 0;
  for (int i = 0; i < L->n_layers; ++i) {
    d.t[i] = L->layer_t[i];
    d.nel[i] = L->layer_nel[i];
    d.z0[i] = z;
    z += L->layer_t[i];
    c += L->layer_nel[i];
    d.cum[i + 1] = c;
  }
  d.nz = c;
  d.T = z;
  d.r_ref = d.radius + 0.5 * d.T;
  d.s_b = 0.25 * M_PI * d.r_ref;
  d.s_a = -d.s_b;
  return d;
}

// Nodes per lattice row and plane: re nodes on a row with even j2 and k2, ro on the other
// rows; pe nodes on a plane of even k2, po on one of odd k2.  A periodic laminate has the
// rows j2 = 0 .. 2 ny - 1 only (j2 = 2 ny is j2 = 0).
__host__ __device__ inline int64_t rows_even(const LamDev& L) { return L.periodic ? L.ny : L.ny + 1; }
__host__ __device__ inline int64_t plane_even(const LamDev& L) {
  return rows_even(L) * (2 * (int64_t)L.nx + 1) + (int64_t)L.ny * ((int64_t)L.nx + 1);
}
__host__ __device__ inline int64_t plane_odd(const LamDev& L) {
  return ((int64_t)L.nx + 1) * rows_even(L);
}

struct Counts {
  int64_t nodes, elems, clamped, faces;
};
static Counts counts(const LamDev& L) {
  Counts k;
  const int64_t nz = L.nz;
  k.nodes = (nz + 1) * plane_even(L) + nz * plane_odd(L);
  k.elems = (int64_t)L.nx * L.ny * nz;
  // nodes on the s = s_min face: 2 ny (+1) on a plane of even k2, ny (+1) on an odd one
  k.clamped = (nz + 1) * (2 * (int64_t)L.ny + (L.periodic ? 0 : 1)) + nz * rows_even(L);
  k.faces = (int64_t)L.ny * nz;
  return k;
}

// node number of lattice point (i2, j2, k2); at most one index is odd
__device__ inline int64_t node_id(const LamDev& L, int i2, int j2, int k2) {
  const int64_t re = 2 * (int64_t)L.nx + 1, ro = (int64_t)L.nx + 1;
  const int64_t pe = plane_even(L), po = plane_odd(L);
  if (L.periodic && j2 == 2 * L.ny) j2 = 0;
  int64_t id = (int64_t)(k2 >> 1) * (pe + po);
  if (k2 & 1) return id + pe + (int64_t)(j2 >> 1) * ro + (i2 >> 1);
  id += (int64_t)(j2 >> 1) * (re + ro);
  if (j2 & 1) return id + re + (i2 >> 1);
  return id + i2;
}

// Boundary i (0..n) of n elements graded with ratio `bias` (largest over smallest element,
// sizes q^e growing geometrically, symmetric about the middle): as a fraction of the
// segment.  e = min(k, n - 1 - k) refines towards both ends, m - e towards the middle
// (m = (n - 1) / 2, q = bias^(1/m)); bias <= 1 gives i / n.
__device__ inline double graded_frac(int i, int n, double bias, bool middle) {
  const int m = (n - 1) / 2;
  if (!(bias > 1.0) || m == 0) return (double)i / n;
  const double q = pow(bias, 1.0 / m);
  double s = 0.0, tot = 0.0;
  for (int k = 0; k < n; ++k) {
    const int e = min(k, n - 1 - k);
    const double h = pow(q, (double)(middle ? m - e : e));
    if (k < i) s += h;
    tot += h;
  }
  return s / tot;
}

__device__ inline double s_bound(const LamDev& L, int i) {
  if (L.geometry == GX_GEOM_FLAT) return L.length * graded_frac(i, L.nx, L.bs, true);
  const int nl = L.nx_limb, na = L.nx - 2 * L.nx_limb;
  if (i <= nl) return L.s_a - L.limb + L.limb * i / nl;
  if (i <= nl + na) return L.s_a + (L.s_b - L.s_a) * graded_frac(i - nl, na, L.bs, true);
  return L.s_b + L.limb * (i - nl - na) / nl;
}

// across the width: uniform strips at both edges, the laminate between graded towards them
__device__ inline double l_bound(const LamDev& L, int j) {
  if (L.strip_ny == 0) return L.width * graded_frac(j, L.ny, L.bl, false);
  const int ns = L.strip_ny;
  const double e = L.strip_w;
  if (j < ns) return e * j / ns;
  if (j > L.ny - ns) return L.width - e + e * (j - (L.ny - ns)) / ns;
  return e + (L.width - 2.0 * e) * graded_frac(j - ns, L.ny - 2 * ns, L.bl, false);
}

__device__ inline double z_bound(const LamDev& L, int k) {
  if (k == 0) return 0.0;
  const int e = k - 1;                           // element layer whose top this is
  int li = 0;
  while (li + 1 < L.n_layers && L.cum[li + 1] <= e) ++li;
  return L.z0[li] + L.t[li] * graded_frac(e - L.cum[li] + 1, L.nel[li], L.bz, false);
}

__device__ inline double lattice(double a, double b, bool odd) {
  return odd ? 0.5 * (a + b) : a;
}

__device__ inline double wrinkle(const LamDev& L, double s) {
  if (L.amp == 0.0) return 0.0;
  const double u = s - (L.geometry == GX_GEOM_FLAT ? 0.5 * L.length : 0.0);
  const double q = u / L.wlen;
  return L.amp * exp(-q * q) * cos(2.0 * M_PI * u / L.wlen);
}

__device__ inline double sech2(double x) {
  const double c = cosh(x);
  return 1.0 / (c * c);
}

// the localised defect of Eq. eq-f as a shift of zeta (0 without one)
__device__ inline double defect(const LamDev& L, double s, double l, double zeta) {
  if (L.dd == 0.0) return 0.0;
  const double sp = 2.0 * (s - L.ds) / L.r_ref;
  const double dz = zeta - L.dz;
  const double b2 = dz < 0 ? L.b2i : L.b2o;
  return L.dd * sech2(sp / L.b1) * sech2(M_PI * dz / (L.radius * b2)) *
         sech2(M_PI * (l - L.dl) / (L.width * L.b3));
}

__device__ inline void map_point(const LamDev& L, double s, double l, double zeta, double* x) {
  const double zh = zeta + wrinkle(L, s) + defect(L, s, l, zeta);
  if (L.geometry == GX_GEOM_FLAT) {
    x[0] = s; x[1] = l; x[2] = zh;
    return;
  }
  const double rho = L.radius + zh;
  x[1] = l;
  if (s < L.s_a) {
    x[0] = L.limb + (s - L.s_a);
    x[2] = rho;
  } else if (s > L.s_b) {
    x[0] = L.limb + rho;
    x[2] = -(s - L.s_b);
  } else {
    const double th = (s - L.s_a) / L.r_ref;
    x[0] = L.limb + rho * sin(th);
    x[2] = rho * cos(th);
  }
}

// lattice parameters (s, l, zeta) of node n
__device__ inline void node_param(const LamDev& L, int64_t n, double* s, double* l,
                                  double* z) {
  const int64_t re = 2 * (int64_t)L.nx + 1, ro = (int64_t)L.nx + 1;
  const int64_t pe = plane_even(L), po = plane_odd(L);
  const int64_t kp = n / (pe + po);
  int64_t rem = n - kp * (pe + po);
  int i2, j2, k2;
  if (rem < pe) {
    k2 = (int)(2 * kp);
    const int64_t jp = rem / (re + ro);
    const int64_t r2 = rem - jp * (re + ro);
    if (r2 < re) { j2 = (int)(2 * jp); i2 = (int)r2; }
    else { j2 = (int)(2 * jp + 1); i2 = (int)(2 * (r2 - re)); }
  } else {
    k2 = (int)(2 * kp + 1);
    rem -= pe;
    j2 = (int)(2 * (rem / ro));
    i2 = (int)(2 * (rem % ro));
  }
  *s = lattice(s_bound(L, i2 >> 1), s_bound(L, (i2 >> 1) + (i2 & 1)), i2 & 1);
  *l = lattice(l_bound(L, j2 >> 1), l_bound(L, (j2 >> 1) + (j2 & 1)), j2 & 1);
  *z = lattice(z_bound(L, k2 >> 1), z_bound(L, (k2 >> 1) + (k2 & 1)), k2 & 1);
}

__global__ void k_nodes(LamDev L, int64_t n_nodes, double* xyz) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_nodes) return;
  double s, l, z;
  node_param(L, n, &s, &l, &z);
  double x[3];
  map_point(L, s, l, z, x);
  xyz[3 * n + 0] = x[0];
  xyz[3 * n + 1] = x[1];
  xyz[3 * n + 2] = x[2];
}

// dX/dp of every node for p = wrinkle amplitude (param 0) or wavelength (param 1): the
// wrinkle shifts zeta_hat = zeta + w(s), so dX/dp = (dX/dzeta_hat) dw/dp, in closed form
__global__ void k_node_velocity(LamDev L, int param, int64_t n_nodes, double* xd) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_nodes) return;
  double s, l, z;
  node_param(L, n, &s, &l, &z);
  const double u = s - (L.geometry == GX_GEOM_FLAT ? 0.5 * L.length : 0.0);
  const double q = u / L.wlen, ph = 2.0 * M_PI * u / L.wlen, g = exp(-q * q);
  const double dw = param == 0 ? g * cos(ph)
                               : L.amp * g * (2.0 * q * u / (L.wlen * L.wlen) * cos(ph) +
                                              sin(ph) * 2.0 * M_PI * u / (L.wlen * L.wlen));
  double d0 = 0.0, d2 = 1.0;                     // dX/dzeta_hat (the y component is 0)
  if (L.geometry != GX_GEOM_FLAT) {
    if (s > L.s_b) { d0 = 1.0; d2 = 0.0; }
    else if (s >= L.s_a) {
      const double th = (s - L.s_a) / L.r_ref;
      d0 = sin(th);
      d2 = cos(th);
    }
  }
  xd[3 * n + 0] = d0 * dw;
  xd[3 * n + 1] = 0.0;
  xd[3 * n + 2] = d2 * dw;
}

// 1 for the elements of the objective region: every element of a flat laminate; the
// elements of the arc (centre of the element's s-range in [s_a, s_b]) of an L-section
__global__ void k_arc_mask(LamDev L, int64_t n_elems, uint8_t* mask) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  const int ex = (int)(e % L.nx);
  const double sc = 0.5 * (s_bound(L, ex) + s_bound(L, ex + 1));
  mask[e] = (L.geometry == GX_GEOM_FLAT || (sc >= L.s_a && sc <= L.s_b)) ? 1 : 0;
}

// lattice offsets (0..2 per axis) of the 20 element nodes in element-local order
__constant__ int8_t c_loc[20][3] = {
    {0, 0, 0}, {2, 0, 0}, {0, 2, 0}, {2, 2, 0}, {0, 0, 2}, {2, 0, 2}, {0, 2, 2}, {2, 2, 2},
    {1, 0, 0}, {1, 2, 0}, {1, 0, 2}, {1, 2, 2},
    {0, 1, 0}, {2, 1, 0}, {0, 1, 2}, {2, 1, 2},
    {0, 0, 1}, {2, 0, 1}, {0, 2, 1}, {2, 2, 1}};

__global__ void k_elems(LamDev L, int64_t n_elems, int32_t* conn, int32_t* elayer) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  const int ex = (int)(e % L.nx);
  const int ey = (int)((e / L.nx) % L.ny);
  const int ez = (int)(e / ((int64_t)L.nx * L.ny));
  for (int a = 0; a < 20; ++a)
    conn[20 * e + a] =
        (int32_t)node_id(L, 2 * ex + c_loc[a][0], 2 * ey + c_loc[a][1], 2 * ez + c_loc[a][2]);
  int li = 0;
  while (li + 1 < L.n_layers && L.cum[li + 1] <= ez) ++li;
  // material overrides: the edge strips, then the stiff end column of the loaded limb
  if (L.strip_ny > 0 && (ey < L.strip_ny || ey >= L.ny - L.strip_ny)) li = L.strip_mat;
  if (L.end_column && ex == L.nx - 1) li = L.end_mat;
  elayer[e] = li;
}

__global__ void k_clamped(LamDev L, int64_t n, int32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t ne = 2 * (int64_t)L.ny + (L.periodic ? 0 : 1);   // even plane's face nodes
  const int64_t per = ne + rows_even(L);                           // per plane pair
  const int64_t kp = i / per, r = i - kp * per;
  int k2, j2;
  if (r < ne) { k2 = (int)(2 * kp); j2 = (int)r; }
  else { k2 = (int)(2 * kp + 1); j2 = (int)(2 * (r - ne)); }
  out[i] = (int32_t)node_id(L, 0, j2, k2);
}

// bit a of wrap[e]: element node a stands for the lattice plane j2 = 2 ny of a periodic
// laminate (its coordinates are those of the node at j2 = 0 plus the width along l)
__global__ void k_wrap(LamDev L, int64_t n_elems, uint32_t* wrap) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  const int ey = (int)((e / L.nx) % L.ny);
  uint32_t m = 0;
  if (L.periodic && ey == L.ny - 1)
    for (int a = 0; a < 20; ++a)
      if (c_loc[a][1] == 2) m |= 1u << a;
  wrap[e] = m;
}

__global__ void k_faces(LamDev L, int64_t n, int32_t* fe, int32_t* fid) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  if (fe) fe[f] = (int32_t)(f * L.nx + (L.nx - 1));
  if (fid) fid[f] = 1;
}

__global__ void k_partition(LamDev L, int64_t n_elems, int px, int py, int32_t* part) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elems) return;
  const int ex = (int)(e % L.nx);
  const int ey = (int)((e / L.nx) % L.ny);
  int ix = 0, iy = 0;
  while (ix + 1 < px && (int64_t)(ix + 1) * L.nx / px <= ex) ++ix;
  while (iy + 1 < py && (int64_t)(iy + 1) * L.ny / py <= ey) ++iy;
  part[e] = iy * px + ix;
}

void laminate_velocity(const gx_laminate* lam, int param, double* xd, hipStream_t st) {
  LamDev L = make_lam(lam);
  GX_REQUIRE(lam->wrinkle_len > 0, "shape derivatives need a wrinkle wavelength > 0");
  Counts k = counts(L);
  hipLaunchKernelGGL(k_node_velocity, dim3(nblocks(k.nodes, 256)), dim3(256), 0, st, L, param,
                     k.nodes, xd);
  GX_HIP(hipGetLastError());
}

void laminate_region(const gx_laminate* lam, uint8_t* mask, hipStream_t st) {
  LamDev L = make_lam(lam);
  Counts k = counts(L);
  hipLaunchKernelGGL(k_arc_mask, dim3(nblocks(k.elems, 256)), dim3(256), 0, st, L, k.elems,
                     mask);
  GX_HIP(hipGetLastError());
}

void laminate_sizes(const gx_laminate* lam, int64_t* n_nodes, int64_t* n_elems) {
  LamDev L = make_lam(lam);
  Counts k = counts(L);
  *n_nodes = k.nodes;
  *n_elems = k.elems;
}

}  // namespace gx

using namespace gx;

extern "C" {

gx_status gx_laminate_counts(const gx_laminate* lam, int64_t* n_nodes, int64_t* n_elems,
                             int64_t* n_clamped, int64_t* n_faces) {
  try {
    LamDev L = make_lam(lam);
    Counts k = counts(L);
    GX_REQUIRE(k.nodes < ((int64_t)1 << 31) / 3, "mesh too large for 32-bit DOF indices");
    if (n_nodes) *n_nodes = k.nodes;
    if (n_elems) *n_elems = k.elems;
    if (n_clamped) *n_clamped = k.clamped;
    if (n_faces) *n_faces = k.faces;
  } catch (const gx::Error& e) {
    return e.code;
  }
  return GX_OK;
}

gx_status gx_laminate_mesh(gx_ctx* c, const gx_laminate* lam, double* xyz, int32_t* conn,
                           int32_t* elem_layer, int32_t* clamped, int32_t* face_elem,
                           int32_t* face_id) {
  GX_API_BEGIN(c)
  LamDev L = make_lam(lam);
  Counts k = counts(L);
  GX_REQUIRE(xyz && conn && elem_layer, "null mesh output");
  hipLaunchKernelGGL(k_nodes, dim3(nblocks(k.nodes, 256)), dim3(256), 0, c->stream, L,
                     k.nodes, xyz);
  hipLaunchKernelGGL(k_elems, dim3(nblocks(k.elems, 256)), dim3(256), 0, c->stream, L,
                     k.elems, conn, elem_layer);
  if (clamped)
    hipLaunchKernelGGL(k_clamped, dim3(nblocks(k.clamped, 256)), dim3(256), 0, c->stream, L,
                       k.clamped, clamped);
  if (face_elem || face_id)
    hipLaunchKernelGGL(k_faces, dim3(nblocks(k.faces, 256)), dim3(256), 0, c->stream, L,
                       k.faces, face_elem, face_id);
  GX_HIP(hipGetLastError());
  GX_HIP(hipStreamSynchronize(c->stream));
  GX_API_END(c)
}

gx_status gx_laminate_wrap(gx_ctx* c, const gx_laminate* lam, uint32_t* elem_wrap) {
  GX_API_BEGIN(c)
  LamDev L = make_lam(lam);
  GX_REQUIRE(elem_wrap, "null wrap output");
  Counts k = counts(L);
  hipLaunchKernelGGL(k_wrap, dim3(nblocks(k.elems, 256)), dim3(256), 0, c->stream, L, k.elems,
                     elem_wrap);
  GX_HIP(hipGetLastError());
  GX_HIP(hipStreamSynchronize(c->stream));
  GX_API_END(c)
}

gx_status gx_laminate_partition(gx_ctx* c, const gx_laminate* lam, int32_t px, int32_t py,
                                int32_t* part) {
  GX_API_BEGIN(c)
  LamDev L = make_lam(lam);
  GX_REQUIRE(px >= 1 && py >= 1 && px <= L.nx && py <= L.ny, "px, py out of range");
  GX_REQUIRE(part, "null partition output");
  Counts k = counts(L);
  hipLaunchKernelGGL(k_partition, dim3(nblocks(k.elems, 256)), dim3(256), 0, c->stream, L,
                     k.elems, px, py, part);
  GX_HIP(hipGetLastError());
  GX_HIP(hipStreamSynchronize(c->stream));
  GX_API_END(c)
}

gx_status gx_laminate_traction(const gx_laminate* lam, int32_t kind, const double* value,
                               gx_traction* out) {
  try {
    LamDev L = make_lam(lam);
    GX_REQUIRE(out && value, "null argument");
    std::memset(out, 0, sizeof(*out));
    if (kind == 0) {
      for (int i = 0; i < 3; ++i) out->t0[i] = value[i];
      return GX_OK;
    }
    GX_REQUIRE(kind == 1, "kind must be 0 (traction) or 1 (moment)");
    const double T = L.T;
    out->k = -12.0 * value[0] / (T * T * T);
    double w_end;
    if (L.geometry == GX_GEOM_FLAT) {
      const double u = 0.5 * L.length;
      w_end = L.amp == 0.0 ? 0.0
                           : L.amp * std::exp(-(u / L.wlen) * (u / L.wlen)) *
                                 std::cos(2.0 * M_PI * u / L.wlen);
      out->c[0] = L.length;
      out->c[2] = 0.5 * T + w_end;
      out->d[2] = 1.0;
    } else {
      const double u = L.s_b + L.limb;
      w_end = L.amp == 0.0 ? 0.0
                           : L.amp * std::exp(-(u / L.wlen) * (u / L.wlen)) *
                                 std::cos(2.0 * M_PI * u / L.wlen);
      out->c[0] = L.limb + L.radius + 0.5 * T + w_end;
      out->c[2] = -L.limb;
      out->d[0] = 1.0;
    }
  } catch (const gx::Error& e) {
    return e.code;
  }
  return GX_OK;
}

}  // extern "C"
