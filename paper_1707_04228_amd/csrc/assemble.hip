// Assembly of K and f (Eq. eq-1) for 20-node serendipity hexahedra with full 3x3x3 Gauss
// integration (section 2.1), and the 3x3-block CSR product y = K x.
//
// Pipeline (all on the device):
//   1. node -> element incidence (counting sort, each list sorted by element number);
//   2. block-CSR pattern: per node, the sorted union of the nodes of its elements;
//   3. material stiffness of each layer from engineering constants (C = S^-1, Table 1);
//   4. element matrices K_e = sum_q B^T C_q B det J w, one work-group per element, with the
//      reference shape-function gradients staged in LDS and C rotated at every Gauss
//      point into the geometric frame and the ply angle by the Bond strain transformation;
//   5. deterministic gather: every block row sums its elements' blocks in element order
//      (no floating-point atomics), then clamped DOFs become identity rows / columns;
//   6. consistent face loads from a 3x3 Gauss rule on each loaded face.
#include <algorithm>
#include <cmath>

#include "element.h"
#include "gx_internal.h"

namespace gx {

constexpr int MAX_ADJ = 32;        // elements sharing one node
constexpr int MAX_ROW = 128;       // blocks in one block row of K

// ---------------------------------------------------------------------------------------
// 1. node -> element incidence
__global__ void k_ne_count(const int32_t* conn, int64_t n_elems, int32_t* cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_elems * 20) return;
  atomicAdd(&cnt[conn[i]], 1);
}
__global__ void k_ne_fill(const int32_t* conn, int64_t n_elems, const int32_t* ptr,
                          int32_t* cursor, int32_t* idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_elems * 20) return;
  const int n = conn[i];
  const int pos = atomicAdd(&cursor[n], 1);
  idx[ptr[n] + pos] = (int32_t)(i / 20);
}
__global__ void k_ne_sort(int64_t n_nodes, const int32_t* ptr, int32_t* idx, int* err) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_nodes) return;
  const int b = ptr[n], e = ptr[n + 1];
  if (e - b > MAX_ADJ) { atomicOr(err, 1); return; }
  if (e == b) atomicOr(err, 2);
  for (int i = b + 1; i < e; ++i) {              // insertion sort (short lists)
    const int v = idx[i];
    int j = i - 1;
    while (j >= b && idx[j] > v) { idx[j + 1] = idx[j]; --j; }
    idx[j + 1] = v;
  }
}

void build_node_elem(gx_ctx* c) {
  const int64_t N = c->n_nodes, E = c->n_elems;
  c->ne_ptr.alloc(N + 1);
  DevBuf<int32_t> cur(N);
  DevBuf<int> err(1);
  DevBuf<int64_t> tmp(scan_tmp_size(N + 1));
  zero(c->ne_ptr, c->stream);
  zero(cur, c->stream);
  zero(err, c->stream);
  hipLaunchKernelGGL(k_ne_count, dim3(nblocks(E * 20, 256)), dim3(256), 0, c->stream,
                     c->conn.p, E, c->ne_ptr.p);
  const int64_t tot = exclusive_scan32(c->ne_ptr.p, N + 1, tmp.p, c->stream);
  GX_REQUIRE(tot == E * 20, "incidence count mismatch");
  c->ne_idx.alloc(E * 20);
  hipLaunchKernelGGL(k_ne_fill, dim3(nblocks(E * 20, 256)), dim3(256), 0, c->stream,
                     c->conn.p, E, c->ne_ptr.p, cur.p, c->ne_idx.p);
  hipLaunchKernelGGL(k_ne_sort, dim3(nblocks(N, 256)), dim3(256), 0, c->stream, N,
                     c->ne_ptr.p, c->ne_idx.p, err.p);
  GX_HIP(hipGetLastError());
  int h = 0;
  to_host(&h, err.p, 1, c->stream);
  GX_REQUIRE(!(h & 1), "a node is shared by more than 32 elements");
  GX_REQUIRE(!(h & 2), "a node belongs to no element");
}

// ---------------------------------------------------------------------------------------
// 2. block-CSR pattern, one 64-lane work-group per node
__device__ inline void bitonic_sort(int32_t* s, int n) {
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const int32_t a = s[i], b = s[l];
          if ((a > b) == up) { s[i] = b; s[l] = a; }
        }
      }
      __syncthreads();
    }
  }
}

// fill == nullptr: count unique neighbours into row_len; else write them at fill + ptr[n]
__global__ void __launch_bounds__(64) k_pattern(const int32_t* conn, const int32_t* ne_ptr,
                                                const int32_t* ne_idx, int32_t* row_len,
                                                const int32_t* ptr, int32_t* fill,
                                                int* err) {
  __shared__ int32_t s[MAX_ADJ * 32];
  __shared__ int32_t wsum[64];
  const int64_t n = blockIdx.x;
  const int b = ne_ptr[n], e = ne_ptr[n + 1];
  const int cnt = (e - b) * 20;
  int sz = 1;
  while (sz < cnt) sz <<= 1;
  for (int i = threadIdx.x; i < sz; i += 64)
    s[i] = i < cnt ? conn[(int64_t)ne_idx[b + i / 20] * 20 + i % 20] : 0x7fffffff;
  __syncthreads();
  bitonic_sort(s, sz);
  // each lane owns a contiguous chunk; count first occurrences
  const int chunk = (sz + 63) / 64;
  const int lo = threadIdx.x * chunk, hi = min(sz, lo + chunk);
  int mine = 0;
  for (int i = lo; i < hi; ++i)
    mine += (s[i] != 0x7fffffff) && (i == 0 || s[i] != s[i - 1]);
  wsum[threadIdx.x] = mine;
  __syncthreads();
  if (fill == nullptr) {
    if (threadIdx.x == 0) {
      int t = 0;
      for (int i = 0; i < 64; ++i) t += wsum[i];
      if (t > MAX_ROW) atomicOr(err, 1);
      row_len[n] = t;
    }
    return;
  }
  int before = 0;
  for (int i = 0; i < (int)threadIdx.x; ++i) before += wsum[i];
  int32_t* out = fill + ptr[n] + before;
  for (int i = lo; i < hi; ++i)
    if ((s[i] != 0x7fffffff) && (i == 0 || s[i] != s[i - 1])) *out++ = s[i];
}

// ---------------------------------------------------------------------------------------
// 3. layer stiffness C = S^-1 from engineering constants (Voigt 11,22,33,23,13,12 with
//    engineering shear strains).  The orthotropic compliance is block diagonal: the normal
//    3x3 block is inverted by cofactors, the shear block is diag(1/G23, 1/G13, 1/G12).
__global__ void k_layer_stiffness(int n_layers, const double* eng, double* C, int* err) {
  const int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= n_layers) return;
  const double* p = eng + 9 * L;
  double E1 = p[0], E2 = p[1], E3 = p[2], G12 = p[3], G13 = p[4], G23 = p[5];
  double n12 = p[6], n13 = p[7], n23 = p[8];
  if (!(G12 > 0)) {                              // isotropic layer given as (E, nu)
    E2 = E3 = E1;
    n13 = n23 = n12;
    G12 = G13 = G23 = E1 / (2.0 * (1.0 + n12));
  }
  const double s11 = 1 / E1, s22 = 1 / E2, s33 = 1 / E3;
  const double s12 = -n12 / E1, s13 = -n13 / E1, s23 = -n23 / E2;
  const double c11 = s22 * s33 - s23 * s23, c22 = s11 * s33 - s13 * s13,
               c33 = s11 * s22 - s12 * s12;
  const double c12 = s13 * s23 - s12 * s33, c13 = s12 * s23 - s13 * s22,
               c23 = s12 * s13 - s11 * s23;
  const double det = s11 * c11 + s12 * c12 + s13 * c13;
  if (!(det > 0) || !(G12 > 0) || !(G13 > 0) || !(G23 > 0) || !(E1 > 0) || !(E2 > 0) ||
      !(E3 > 0)) {
    atomicOr(err, 1);
    return;
  }
  double* o = C + 36 * L;
  for (int i = 0; i < 36; ++i) o[i] = 0.0;
  o[0] = c11 / det; o[7] = c22 / det; o[14] = c33 / det;
  o[1] = o[6] = c12 / det;
  o[2] = o[12] = c13 / det;
  o[8] = o[13] = c23 / det;
  o[21] = G23; o[28] = G13; o[35] = G12;
}

// ---------------------------------------------------------------------------------------
// 4. element stiffness, one 256-thread work-group per element (grid-stride)
struct ElemSmem {
  double dNr[27][20][3];     // reference gradients at the Gauss points
  double X[20][3];
  double G[27][20][3];       // physical gradients
  double Cg[27][36];         // rotated stiffness
  double dv[27];             // det J * weight
  double CB[20][6][3];       // C_q B_b for the current Gauss point
};

// strain-displacement entry B_a[I][i] (Voigt row I, displacement component i) from g = grad N_a
__device__ inline double bent(int I, int i, const double* g) {
  // rows: 0 e11, 1 e22, 2 e33, 3 g23, 4 g13, 5 g12
  switch (I) {
    case 0: return i == 0 ? g[0] : 0.0;
    case 1: return i == 1 ? g[1] : 0.0;
    case 2: return i == 2 ? g[2] : 0.0;
    case 3: return i == 1 ? g[2] : (i == 2 ? g[1] : 0.0);
    case 4: return i == 0 ? g[2] : (i == 2 ? g[0] : 0.0);
    default: return i == 0 ? g[1] : (i == 1 ? g[0] : 0.0);
  }
}

__device__ inline void gauss_point_setup(int q, const ElemSmem& sm, const double* Cl,
                                         double angle, double* Gout, double* Cgout,
                                         double* dvout, int* bad) {
  // Jacobian J[i][j] = dx_i / dxi_j
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int a = 0; a < 20; ++a)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) J[i][j] += sm.X[a][i] * sm.dNr[q][a][j];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  if (!(det > 0)) *bad = 1;
  const double id = 1.0 / det;
  double Ji[3][3];                               // Ji[j][i] = dxi_j / dx_i
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  for (int a = 0; a < 20; ++a)
    for (int i = 0; i < 3; ++i)
      Gout[3 * a + i] = sm.dNr[q][a][0] * Ji[0][i] + sm.dNr[q][a][1] * Ji[1][i] +
                        sm.dNr[q][a][2] * Ji[2][i];
  // geometric frame: e1 along dx/dxi, e2 from dx/deta (Gram-Schmidt), e3 = e1 x e2
  double e1[3] = {J[0][0], J[1][0], J[2][0]}, t2[3] = {J[0][1], J[1][1], J[2][1]};
  const double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int i = 0; i < 3; ++i) e1[i] /= n1;
  const double pr = t2[0] * e1[0] + t2[1] * e1[1] + t2[2] * e1[2];
  double e2[3] = {t2[0] - pr * e1[0], t2[1] - pr * e1[1], t2[2] - pr * e1[2]};
  const double n2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
  for (int i = 0; i < 3; ++i) e2[i] /= n2;
  const double e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
  // material axes (rows of Q, global components): fibre rotated by the ply angle about e3
  const double ca = cos(angle), sa = sin(angle);
  double Q[3][3];
  for (int i = 0; i < 3; ++i) {
    Q[0][i] = ca * e1[i] + sa * e2[i];
    Q[1][i] = -sa * e1[i] + ca * e2[i];
    Q[2][i] = e3[i];
  }
  // Bond matrix: local engineering strain = T * global engineering strain
  const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
  double T[6][6];
  for (int I = 0; I < 6; ++I) {
    const int i = vi[I], j = vj[I];
    for (int K = 0; K < 6; ++K) {
      const int k = vi[K], l = vj[K];
      if (I < 3)
        T[I][K] = (K < 3) ? Q[i][k] * Q[i][k] : Q[i][k] * Q[i][l];
      else
        T[I][K] = (K < 3) ? 2.0 * Q[i][k] * Q[j][k] : Q[i][k] * Q[j][l] + Q[i][l] * Q[j][k];
    }
  }
  // C_g = T^T C T
  double CT[6][6];
  for (int I = 0; I < 6; ++I)
    for (int K = 0; K < 6; ++K) {
      double s = 0;
      for (int L = 0; L < 6; ++L) s += Cl[6 * I + L] * T[L][K];
      CT[I][K] = s;
    }
  for (int I = 0; I < 6; ++I)
    for (int K = I; K < 6; ++K) {
      double s = 0;
      for (int L = 0; L < 6; ++L) s += T[L][I] * CT[L][K];
      Cgout[6 * I + K] = s;
      Cgout[6 * K + I] = s;
    }
  double xq, wq, yq, wy, zq, wz;
  gauss3(q % 3, &xq, &wq);
  gauss3((q / 3) % 3, &yq, &wy);
  gauss3(q / 9, &zq, &wz);
  *dvout = det * wq * wy * wz;
}

__global__ void __launch_bounds__(256) k_element(Periodic P, int64_t n_elems, const double* xyz,
                                                 const int32_t* conn, const int32_t* elayer,
                                                 const double* Clayer, const double* angle,
                                                 double* Ke, int* err) {
  extern __shared__ double smem_raw[];
  ElemSmem& sm = *reinterpret_cast<ElemSmem*>(smem_raw);
  const int t = threadIdx.x;
  // reference gradients at the 27 Gauss points (q = i + 3 j + 9 k)
  for (int idx = t; idx < 27 * 20; idx += blockDim.x) {
    const int q = idx / 20, a = idx % 20;
    double x0, x1, x2, w;
    gauss3(q % 3, &x0, &w);
    gauss3((q / 3) % 3, &x1, &w);
    gauss3(q / 9, &x2, &w);
    double N, d[3];
    shape_one(a, x0, x1, x2, &N, d);
    sm.dNr[q][a][0] = d[0];
    sm.dNr[q][a][1] = d[1];
    sm.dNr[q][a][2] = d[2];
  }
  // node pair (pa <= pb) owned by this thread
  int pa = -1, pb = -1;
  if (t < 210) {
    int r = t, a = 0;
    while (r >= 20 - a) { r -= 20 - a; ++a; }
    pa = a;
    pb = a + r;
  }
  __syncthreads();
  for (int64_t e = blockIdx.x; e < n_elems; e += gridDim.x) {
    if (t < 60) sm.X[t / 3][t % 3] = node_coord(xyz, conn[20 * e + t / 3], t % 3, P, e, t / 3);
    __syncthreads();
    const int L = elayer[e];
    if (t < 27) {
      int bad = 0;
      gauss_point_setup(t, sm, Clayer + 36 * L, angle[L] * (M_PI / 180.0), &sm.G[t][0][0],
                        &sm.Cg[t][0], &sm.dv[t], &bad);
      if (bad) atomicOr(err, 1);
    }
    __syncthreads();
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = 0; q < 27; ++q) {
      if (t < 60) {                                // C_q B_b, node b, component k
        const int b = t / 3, k = t % 3;
        const double* g = sm.G[q][b];
        for (int I = 0; I < 6; ++I) {
          double s = 0;
          for (int J = 0; J < 6; ++J) s += sm.Cg[q][6 * I + J] * bent(J, k, g);
          sm.CB[b][I][k] = s;
        }
      }
      __syncthreads();
      if (pa >= 0) {
        const double* g = sm.G[q][pa];
        const double dv = sm.dv[q];
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) {
            double s = 0;
            for (int I = 0; I < 6; ++I) s += bent(I, i, g) * sm.CB[pb][I][k];
            acc[3 * i + k] += dv * s;
          }
      }
      __syncthreads();
    }
    if (pa >= 0) {
      double* out = Ke + (((int64_t)e * 20 + pa) * 20 + pb) * 9;
      for (int i = 0; i < 9; ++i) out[i] = acc[i];
      if (pa != pb) {
        double* o2 = Ke + (((int64_t)e * 20 + pb) * 20 + pa) * 9;
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) o2[3 * k + i] = acc[3 * i + k];
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// 5. deterministic gather of element blocks into block rows; clamped DOFs -> identity
__global__ void __launch_bounds__(64) k_gather(const int32_t* conn, const int32_t* ne_ptr,
                                               const int32_t* ne_idx, const int32_t* row_ptr,
                                               const int32_t* col, const double* Ke,
                                               const uint8_t* fixed, double* val) {
  __shared__ double rv[MAX_ROW * 9];
  __shared__ int32_t rc[MAX_ROW];
  const int64_t n = blockIdx.x;
  const int rb = row_ptr[n], len = row_ptr[n + 1] - rb;
  for (int i = threadIdx.x; i < len; i += 64) rc[i] = col[rb + i];
  for (int i = threadIdx.x; i < len * 9; i += 64) rv[i] = 0.0;
  __syncthreads();
  for (int k = ne_ptr[n]; k < ne_ptr[n + 1]; ++k) {
    const int64_t e = ne_idx[k];
    int a = 0;
    while (conn[20 * e + a] != n) ++a;
    for (int v = threadIdx.x; v < 180; v += 64) {
      const int b = v / 9, comp = v - 9 * (v / 9);
      const int m = conn[20 * e + b];
      int lo = 0, hi = len - 1;                  // binary search of m in the row
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rc[mid] < m) lo = mid + 1; else hi = mid;
      }
      rv[9 * lo + comp] += Ke[((e * 20 + a) * 20 + b) * 9 + comp];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < len * 9; i += 64) {
    const int blk = i / 9, comp = i - 9 * (i / 9);
    const int ri = comp / 3, ci = comp - 3 * (comp / 3);
    const int64_t rd = 3 * n + ri, cd = 3 * (int64_t)rc[blk] + ci;
    double v = rv[i];
    if (fixed[rd] || fixed[cd]) v = (rd == cd) ? 1.0 : 0.0;
    val[(int64_t)rb * 9 + i] = v;
  }
}

// ---------------------------------------------------------------------------------------
// 6. consistent face loads; t = t0 + k ((x - c) . d) n_out, 3x3 Gauss rule on the face;
//    one thread per (face, element node) writes its three components to fl; k_face_gather
//    then sums each node's entries in a fixed order (face, then local node), so f is the
//    same bit for bit on every run
__global__ void k_face_loads(Periodic P, int64_t n_faces, const int32_t* fe, const int32_t* fid,
                             const double* xyz, const int32_t* conn, gx_traction tr,
                             double* fl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_faces * 20) return;
  const int64_t e = fe[idx / 20];
  const int na = (int)(idx % 20);
  const int face = fid[idx / 20];
  const int ax = face / 2;
  const double sgn = (face & 1) ? 1.0 : -1.0;
  double fl0 = 0, fl1 = 0, fl2 = 0;
  for (int qb = 0; qb < 3; ++qb)
    for (int qc = 0; qc < 3; ++qc) {
      double pb, wb, pc, wc;
      gauss3(qb, &pb, &wb);
      gauss3(qc, &pc, &wc);
      // reference point on the face: fixed axis ax, in-face axes (ax+1)%3, (ax+2)%3
      const double p0 = ax == 0 ? sgn : (ax == 1 ? pc : pb);
      const double p1 = ax == 1 ? sgn : (ax == 2 ? pc : pb);
      const double p2 = ax == 2 ? sgn : (ax == 0 ? pc : pb);
      double x0 = 0, x1 = 0, x2 = 0, tb0 = 0, tb1 = 0, tb2 = 0, tc0 = 0, tc1 = 0, tc2 = 0,
             Na = 0;
      for (int a = 0; a < 20; ++a) {
        double N, d[3];
        shape_one(a, p0, p1, p2, &N, d);
        const double db = ax == 0 ? d[1] : (ax == 1 ? d[2] : d[0]);
        const double dc = ax == 0 ? d[2] : (ax == 1 ? d[0] : d[1]);
        const int64_t nd = conn[20 * e + a];
        const double X0 = node_coord(xyz, nd, 0, P, e, a), X1 = node_coord(xyz, nd, 1, P, e, a),
                     X2 = node_coord(xyz, nd, 2, P, e, a);
        x0 += N * X0; x1 += N * X1; x2 += N * X2;
        tb0 += db * X0; tb1 += db * X1; tb2 += db * X2;
        tc0 += dc * X0; tc1 += dc * X1; tc2 += dc * X2;
        if (a == na) Na = N;
      }
      const double nv0 = tb1 * tc2 - tb2 * tc1, nv1 = tb2 * tc0 - tb0 * tc2,
                   nv2 = tb0 * tc1 - tb1 * tc0;
      const double dA = sqrt(nv0 * nv0 + nv1 * nv1 + nv2 * nv2);
      const double lin = tr.k * ((x0 - tr.c[0]) * tr.d[0] + (x1 - tr.c[1]) * tr.d[1] +
                                 (x2 - tr.c[2]) * tr.d[2]);
      const double w = wb * wc * dA * Na;
      fl0 += (tr.t0[0] + lin * sgn * nv0 / dA) * w;
      fl1 += (tr.t0[1] + lin * sgn * nv1 / dA) * w;
      fl2 += (tr.t0[2] + lin * sgn * nv2 / dA) * w;
    }
  fl[3 * idx] = fl0;
  fl[3 * idx + 1] = fl1;
  fl[3 * idx + 2] = fl2;
}

// f at the loaded nodes: node unode[i] sums the entries uidx[uptr[i] .. uptr[i + 1]) of fl
// (ascending (face, local node) order); clamped components stay zero
__global__ void k_face_gather(int64_t n_unique, const int32_t* uptr, const int32_t* uidx,
                              const int32_t* unode, const double* fl, const uint8_t* fixed,
                              double* f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_unique) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int32_t k = uptr[i]; k < uptr[i + 1]; ++k) {
    const int64_t j = uidx[k];
    a0 += fl[3 * j];
    a1 += fl[3 * j + 1];
    a2 += fl[3 * j + 2];
  }
  const int64_t d = 3 * (int64_t)unode[i];
  f[d] = fixed[d] ? 0.0 : a0;
  f[d + 1] = fixed[d + 1] ? 0.0 : a1;
  f[d + 2] = fixed[d + 2] ? 0.0 : a2;
}

__global__ void k_fixed(int64_t n, const int32_t* nodes, uint8_t* fixed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t d = 3 * (int64_t)nodes[i];
  fixed[d] = fixed[d + 1] = fixed[d + 2] = 1;
}

// ---------------------------------------------------------------------------------------
// y = K x, one 64-lane wavefront per block row.  The values of a row are contiguous, 9 per
// 3x3 block.  Pass u takes the row's blocks 7 u .. 7 u + 6: lane l < 63 reads value
// 63 u + l, i.e. entry l % 9 of block 7 u + l / 9, so every lane multiplies the same
// entry position on every pass and keeps a single sum (the block-row component
// (l % 9) / 3, the x component l % 3), and each pass is one coalesced 504-byte load of
// values.  A row takes ceil(blocks / 7) passes (rounds of 12 past 84 blocks).  All value
// loads of a round are issued; its column indices are loaded once, one block per lane, and
// passed between lanes; then all gathers of x are issued, before the products.  The three
// components are then summed through LDS (lanes 0-2, the 21 sums of their component in a
// fixed order).
constexpr int SPMV_PASSES = 12;                   // 84 blocks per round (rows of the
                                                  // 20-node meshes have at most 81)
__global__ void __launch_bounds__(256) k_spmv(int64_t n_rows, const int32_t* __restrict__ rp,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ val,
                                              const double* __restrict__ x,
                                              double* __restrict__ y) {
  __shared__ double red[4][64];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  // work-groups are dealt to the eight XCDs in turn; each XCD takes a contiguous eighth of
  // the rows, so the part of x its rows gather stays in its L2
  const int64_t xcd = blockIdx.x & 7, nq = gridDim.x >> 3, nrem = gridDim.x & 7;
  const int64_t lb = xcd * nq + min(xcd, nrem) + (blockIdx.x >> 3);
  const int64_t row = lb * 4 + w;                 // uniform: the row bounds are scalar
  if (row >= n_rows) return;                       // whole wavefronts
  const int q = lane / 9, e = lane - 9 * q, c = e % 3;
  const int b0 = rp[row], nb = rp[row + 1] - b0;
  const double* vrow = val + (int64_t)b0 * 9 + e;
  const int32_t* crow = col + b0;
  double acc = 0.0;
  // one round of P passes over blocks k0 ..; lanes past the row's last block repeat it
  // and are masked
  auto round = [&](int k0, auto np) {
    constexpr int P = decltype(np)::value;
    double pv[P], xv[P];
    // the round's column indices, one block per lane (blocks k0 + 64 .. in a second
    // register past 64 blocks); pass u takes block 7 u + q's from its lane
    const int cl0 = crow[min(k0 + lane, nb - 1)];
    const int cl1 = 7 * P > 64 ? crow[min(k0 + 64 + lane, nb - 1)] : 0;
#pragma unroll
    for (int u = 0; u < P; ++u)                   // read once: kept out of the caches' way
      pv[u] = __builtin_nontemporal_load(&vrow[9 * min(k0 + 7 * u + q, nb - 1)]);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int b = 7 * u + q;                     // block within the round (< 84)
      // (a permute reads 0 from an inactive lane, so both run with the whole wavefront
      // active and the block's register is selected afterwards)
      int xi;
      if (7 * u + 6 < 64) {
        xi = __builtin_amdgcn_ds_bpermute(4 * b, cl0);
      } else if (7 * u >= 64) {
        xi = __builtin_amdgcn_ds_bpermute(4 * (b - 64), cl1);
      } else {
        const int i0 = __builtin_amdgcn_ds_bpermute(4 * (b & 63), cl0);
        const int i1 = __builtin_amdgcn_ds_bpermute(4 * (b & 63), cl1);
        xi = b < 64 ? i0 : i1;
      }
      xv[u] = x[3 * (int64_t)xi + c];
    }
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const bool ok = lane < 63 && k0 + 7 * u + q < nb;  // masked, not branched
      acc += ok ? pv[u] * xv[u] : 0.0;
    }
  };
  // exactly the passes the row needs (rounds of SPMV_PASSES past 7 SPMV_PASSES blocks)
  using std::integral_constant;
  switch ((nb + 6) / 7) {
    case 0: break;
    case 1: round(0, integral_constant<int, 1>{}); break;
    case 2: round(0, integral_constant<int, 2>{}); break;
    case 3: round(0, integral_constant<int, 3>{}); break;
    case 4: round(0, integral_constant<int, 4>{}); break;
    case 5: round(0, integral_constant<int, 5>{}); break;
    case 6: round(0, integral_constant<int, 6>{}); break;
    case 7: round(0, integral_constant<int, 7>{}); break;
    case 8: round(0, integral_constant<int, 8>{}); break;
    case 9: round(0, integral_constant<int, 9>{}); break;
    case 10: round(0, integral_constant<int, 10>{}); break;
    case 11: round(0, integral_constant<int, 11>{}); break;
    default:
      for (int k0 = 0; k0 < nb; k0 += 7 * SPMV_PASSES)
        round(k0, integral_constant<int, SPMV_PASSES>{});
  }
  // lanes of one wavefront exchange through LDS without a barrier: its LDS accesses are
  // performed in order
  red[w][lane] = acc;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_wave_barrier();
  if (lane < 3) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 7; ++t)
#pragma unroll
      for (int j = 0; j < 3; ++j) s += red[w][9 * t + 3 * lane + j];
    y[3 * row + lane] = s;
  }
}

void spmv(gx_ctx* c, const double* x, double* y) {
  hipLaunchKernelGGL(k_spmv, dim3(nblocks(c->n_nodes, 4)), dim3(256), 0, c->stream,
                     c->n_nodes, c->row_ptr.p, c->col.p, c->val.p, x, y);
}

}  // namespace gx

using namespace gx;

extern "C" {

gx_status gx_assemble(gx_ctx* c, const gx_mesh* m, const gx_plystack* ps, const gx_loads* ld,
                      double* f_out) {
  GX_API_BEGIN(c)
  GX_REQUIRE(m && ps && ld && f_out, "null argument");
  GX_REQUIRE(m->n_nodes > 0 && m->n_elems > 0 && m->xyz && m->conn && m->elem_layer,
             "bad mesh");
  GX_REQUIRE(m->n_nodes < ((int64_t)1 << 31) / 3, "too many nodes");
  GX_REQUIRE(ps->n_layers >= 1 && ps->eng && ps->angle_deg, "bad ply stack");
  Timer tm(c->stream);
  hipStream_t s = c->stream;
  c->assembled = false;
  c->matrix_only = false;
  c->setup_done = false;
  c->sw = Schwarz();
  c->n_nodes = m->n_nodes;
  c->n_elems = m->n_elems;
  const int64_t N = c->n_nodes, E = c->n_elems;
  c->xyz.alloc(3 * N);
  c->conn.alloc(20 * E);
  c->elayer.alloc(E);
  GX_HIP(hipMemcpyAsync(c->xyz.p, m->xyz, 3 * N * sizeof(double), hipMemcpyDefault, s));
  GX_HIP(hipMemcpyAsync(c->conn.p, m->conn, 20 * E * sizeof(int32_t), hipMemcpyDefault, s));
  GX_HIP(hipMemcpyAsync(c->elayer.p, m->elem_layer, E * sizeof(int32_t), hipMemcpyDefault, s));
  c->wrap.release();
  for (int i = 0; i < 3; ++i) c->period[i] = m->elem_wrap ? m->period[i] : 0.0;
  if (m->elem_wrap) {
    c->wrap.alloc(E);
    GX_HIP(hipMemcpyAsync(c->wrap.p, m->elem_wrap, E * sizeof(uint32_t), hipMemcpyDefault, s));
  }
  std::vector<int32_t> hc(20 * E);                 // host copy of conn (checks, face loads)
  {  // validate indices on the host side of a copy (cheap relative to assembly)
    std::vector<int32_t> hl(E);
    to_host(hc.data(), c->conn.p, 20 * E, s);
    to_host(hl.data(), c->elayer.p, E, s);
    for (int32_t v : hc) GX_REQUIRE(v >= 0 && v < N, "connectivity index out of range");
    for (int32_t v : hl) GX_REQUIRE(v >= 0 && v < ps->n_layers, "layer index out of range");
  }
  // clamped DOFs
  c->fixed.alloc(3 * N);
  zero(c->fixed, s);
  if (ld->n_clamped > 0) {
    GX_REQUIRE(ld->clamped, "null clamped list");
    std::vector<int32_t> h(ld->n_clamped);
    GX_HIP(hipMemcpyAsync(h.data(), ld->clamped, h.size() * sizeof(int32_t), hipMemcpyDefault,
                          s));
    GX_HIP(hipStreamSynchronize(s));
    for (int32_t v : h) GX_REQUIRE(v >= 0 && v < N, "clamped node out of range");
    DevBuf<int32_t> dn(ld->n_clamped);
    to_dev(dn.p, h.data(), h.size(), s);
    hipLaunchKernelGGL(k_fixed, dim3(nblocks(ld->n_clamped, 256)), dim3(256), 0, s,
                       (int64_t)ld->n_clamped, dn.p, c->fixed.p);
    GX_HIP(hipStreamSynchronize(s));
  }
  build_node_elem(c);
  // pattern
  DevBuf<int> err(1);
  zero(err, s);
  c->row_ptr.alloc(N + 1);
  zero(c->row_ptr, s);
  hipLaunchKernelGGL(k_pattern, dim3((unsigned)N), dim3(64), 0, s, c->conn.p, c->ne_ptr.p,
                     c->ne_idx.p, c->row_ptr.p, (const int32_t*)nullptr, (int32_t*)nullptr,
                     err.p);
  GX_HIP(hipGetLastError());
  DevBuf<int64_t> tmp(scan_tmp_size(N + 1));
  const int64_t nnzb = exclusive_scan32(c->row_ptr.p, N + 1, tmp.p, s);
  GX_REQUIRE(nnzb * 9 < ((int64_t)1 << 40), "matrix too large");
  c->nnzb = nnzb;
  c->col.alloc(nnzb);
  hipLaunchKernelGGL(k_pattern, dim3((unsigned)N), dim3(64), 0, s, c->conn.p, c->ne_ptr.p,
                     c->ne_idx.p, (int32_t*)nullptr, c->row_ptr.p, c->col.p, err.p);
  GX_HIP(hipGetLastError());
  int herr = 0;
  to_host(&herr, err.p, 1, s);
  GX_REQUIRE(!herr, "a block row has more than 128 blocks");
  // materials
  DevBuf<double> eng(9 * ps->n_layers);
  DevBuf<double>& ang = c->ang;
  DevBuf<double>& Cl = c->Cl;
  ang.alloc(ps->n_layers);
  Cl.alloc(36 * ps->n_layers);
  c->n_layers = ps->n_layers;
  c->eng.assign(ps->eng, ps->eng + 9 * ps->n_layers);
  to_dev(eng.p, ps->eng, 9 * ps->n_layers, s);
  to_dev(ang.p, ps->angle_deg, ps->n_layers, s);
  hipLaunchKernelGGL(k_layer_stiffness, dim3(nblocks(ps->n_layers, 64)), dim3(64), 0, s,
                     ps->n_layers, eng.p, Cl.p, err.p);
  to_host(&herr, err.p, 1, s);
  GX_REQUIRE(!herr, "singular material compliance");
  // element matrices
  c->Ke.alloc((size_t)E * 3600);
  const unsigned eg = (unsigned)std::min<int64_t>(E, 256 * 32);
  hipLaunchKernelGGL(k_element, dim3(eg), dim3(256), sizeof(ElemSmem), s, periodic_of(c), E, c->xyz.p,
                     c->conn.p, c->elayer.p, Cl.p, ang.p, c->Ke.p, err.p);
  GX_HIP(hipGetLastError());
  to_host(&herr, err.p, 1, s);
  GX_REQUIRE(!herr, "non-positive Jacobian determinant in an element");
  // global matrix
  c->val.alloc((size_t)nnzb * 9);
  hipLaunchKernelGGL(k_gather, dim3((unsigned)N), dim3(64), 0, s, c->conn.p, c->ne_ptr.p,
                     c->ne_idx.p, c->row_ptr.p, c->col.p, c->Ke.p, c->fixed.p, c->val.p);
  GX_HIP(hipGetLastError());
  // loads
  GX_HIP(hipMemsetAsync(f_out, 0, 3 * N * sizeof(double), s));
  c->n_faces = 0;
  if (ld->n_faces > 0) {
    GX_REQUIRE(ld->face_elem && ld->face_id, "null face list");
    std::vector<int32_t> he(ld->n_faces), hf(ld->n_faces);
    GX_HIP(hipMemcpyAsync(he.data(), ld->face_elem, he.size() * 4, hipMemcpyDefault, s));
    GX_HIP(hipMemcpyAsync(hf.data(), ld->face_id, hf.size() * 4, hipMemcpyDefault, s));
    GX_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < ld->n_faces; ++i)
      GX_REQUIRE(he[i] >= 0 && he[i] < E && hf[i] >= 0 && hf[i] < 6, "bad load face");
    DevBuf<int32_t>& de = c->face_e;
    DevBuf<int32_t>& df = c->face_id;
    de.alloc(ld->n_faces);
    df.alloc(ld->n_faces);
    c->n_faces = ld->n_faces;
    c->traction = ld->traction;
    to_dev(de.p, he.data(), he.size(), s);
    to_dev(df.p, hf.data(), hf.size(), s);
    const int64_t nent = ld->n_faces * 20;
    DevBuf<double> fl(3 * nent);
    hipLaunchKernelGGL(k_face_loads, dim3(nblocks(nent, 64)), dim3(64), 0, s, periodic_of(c),
                       (int64_t)ld->n_faces, de.p, df.p, c->xyz.p, c->conn.p, ld->traction,
                       fl.p);
    GX_HIP(hipGetLastError());
    // per node, its (face, local node) entries in ascending order
    std::vector<int32_t> order(nent);
    for (int64_t k = 0; k < nent; ++k) order[k] = (int32_t)k;
    auto node_of = [&](int32_t k) { return hc[20 * (int64_t)he[k / 20] + k % 20]; };
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return node_of(a) < node_of(b); });
    std::vector<int32_t> uptr{0}, unode;
    for (int64_t k = 0; k < nent; ++k) {
      if (k > 0 && node_of(order[k]) != node_of(order[k - 1])) uptr.push_back((int32_t)k);
      if (k == 0 || node_of(order[k]) != node_of(order[k - 1])) unode.push_back(node_of(order[k]));
    }
    uptr.push_back((int32_t)nent);
    DevBuf<int32_t> d_uptr(uptr.size()), d_uidx(nent), d_unode(unode.size());
    to_dev(d_uptr.p, uptr.data(), uptr.size(), s);
    to_dev(d_uidx.p, order.data(), order.size(), s);
    to_dev(d_unode.p, unode.data(), unode.size(), s);
    hipLaunchKernelGGL(k_face_gather, dim3(nblocks((int64_t)unode.size(), 256)), dim3(256), 0, s,
                       (int64_t)unode.size(), d_uptr.p, d_uidx.p, d_unode.p, fl.p, c->fixed.p,
                       f_out);
    GX_HIP(hipGetLastError());
    GX_HIP(hipStreamSynchronize(s));
  }
  GX_HIP(hipStreamSynchronize(s));
  c->assembled = true;
  c->phase_ms[0] = tm.ms();
  GX_API_END(c)
}

gx_status gx_matrix_info(gx_ctx* c, int64_t* nr, int64_t* nb) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "matrix not assembled");
  if (nr) *nr = c->n_nodes;
  if (nb) *nb = c->nnzb;
  GX_API_END(c)
}

gx_status gx_matrix_copy(gx_ctx* c, int32_t* rp, int32_t* col, double* val) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "matrix not assembled");
  hipStream_t s = c->stream;
  if (rp)
    GX_HIP(hipMemcpyAsync(rp, c->row_ptr.p, (c->n_nodes + 1) * 4, hipMemcpyDefault, s));
  if (col) GX_HIP(hipMemcpyAsync(col, c->col.p, c->nnzb * 4, hipMemcpyDefault, s));
  if (val) GX_HIP(hipMemcpyAsync(val, c->val.p, c->nnzb * 72, hipMemcpyDefault, s));
  GX_HIP(hipStreamSynchronize(s));
  GX_API_END(c)
}

gx_status gx_matrix_load(gx_ctx* c, int64_t n_block_rows, int64_t n_blocks,
                         const int32_t* row_ptr, const int32_t* col, const double* val) {
  GX_API_BEGIN(c)
  GX_REQUIRE(n_block_rows >= 1 && n_blocks >= 0 && row_ptr && (col && val || n_blocks == 0),
             "bad block matrix");
  GX_REQUIRE(n_block_rows < ((int64_t)1 << 31) / 3 && n_blocks < ((int64_t)1 << 31),
             "block matrix too large for 32-bit indices");
  hipStream_t s = c->stream;
  std::vector<int32_t> hp(n_block_rows + 1), hc(n_blocks);
  GX_HIP(hipMemcpyAsync(hp.data(), row_ptr, hp.size() * 4, hipMemcpyDefault, s));
  if (n_blocks) GX_HIP(hipMemcpyAsync(hc.data(), col, hc.size() * 4, hipMemcpyDefault, s));
  GX_HIP(hipStreamSynchronize(s));
  GX_REQUIRE(hp[0] == 0 && hp[n_block_rows] == n_blocks, "row pointers do not span the blocks");
  for (int64_t r = 0; r < n_block_rows; ++r) GX_REQUIRE(hp[r] <= hp[r + 1], "row pointers decrease");
  for (int32_t v : hc) GX_REQUIRE(v >= 0 && v < n_block_rows, "column index out of range");
  c->assembled = false;
  c->setup_done = false;
  c->sw = Schwarz();
  c->n_nodes = n_block_rows;
  c->n_elems = 0;
  c->nnzb = n_blocks;
  c->row_ptr.alloc(n_block_rows + 1);
  c->col.alloc(std::max<int64_t>(n_blocks, 1));
  c->val.alloc(std::max<int64_t>(9 * n_blocks, 1));
  to_dev(c->row_ptr.p, hp.data(), hp.size(), s);
  if (n_blocks) {
    to_dev(c->col.p, hc.data(), hc.size(), s);
    GX_HIP(hipMemcpyAsync(c->val.p, val, 9 * n_blocks * sizeof(double), hipMemcpyDefault, s));
  }
  GX_HIP(hipStreamSynchronize(s));
  c->assembled = true;
  c->matrix_only = true;
  GX_API_END(c)
}

gx_status gx_spmv(gx_ctx* c, const double* x, double* y) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "matrix not assembled");
  GX_REQUIRE(x && y, "null vector");
  spmv(c, x, y);
  GX_HIP(hipGetLastError());
  GX_HIP(hipStreamSynchronize(c->stream));
  GX_API_END(c)
}

}  // extern "C"
