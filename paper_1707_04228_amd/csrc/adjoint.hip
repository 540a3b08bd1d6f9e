// Adjoint sensitivities of a through-thickness stress functional (an extension of the
// paper's solver: its corner-unfolding analysis is driven by the through-thickness stress
// sigma_33 in the curved region, section 3).
//
//   J(u, p) = sum over the region's elements and Gauss points of sigma_33(q)^2 det J w,
//
// sigma_33 the normal stress along the laminate normal e3 of the local frame (the third
// material axis).  With K lambda = dJ/du (solved by PCG with the same preconditioner),
//
//   dJ/dp = dJ/dp|_u - lambda^T (dK/dp u - df/dp)
//
// for p = wrinkle amplitude A, wrinkle wavelength L_w (through the node coordinates, whose
// derivatives are closed forms of the wrinkle map) and the modulus E11 of every layer
// (through dC/dE11 = -C (dS/dE11) C).  The element-level derivatives are exact directional
// derivatives: the element routine is evaluated in forward-mode dual numbers along dX/dp or
// dC/dp.  The element strains are rotated into the material frame (eps' = Q eps Q^T), so
// sigma'_3 is the through-thickness stress directly.
#include <cmath>

#include "element.h"
#include "gx_internal.h"

namespace gx {

// ---- forward-mode dual numbers
struct Dual {
  double v, d;
};
__device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
__device__ inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ inline Dual operator/(Dual a, Dual b) {
  const double i = 1.0 / b.v;
  return {a.v * i, (a.d - a.v * b.d * i) * i};
}
__device__ inline Dual& operator+=(Dual& a, Dual b) {
  a.v += b.v;
  a.d += b.d;
  return a;
}
__device__ inline Dual dsqrt(Dual a) {
  const double r = sqrt(a.v);
  return {r, 0.5 * a.d / r};
}
__device__ inline double dsqrt(double a) { return sqrt(a); }
__device__ inline double val(double a) { return a; }
__device__ inline double val(Dual a) { return a.v; }
__device__ inline double der(double) { return 0.0; }
__device__ inline double der(Dual a) { return a.d; }
template <class R> __device__ inline R mk(double v, double d);
template <> __device__ inline double mk<double>(double v, double) { return v; }
template <> __device__ inline Dual mk<Dual>(double v, double d) { return {v, d}; }

struct SensArgs {
  Periodic P;
  const double* xyz;
  const double* xd;          // dX/dp per node (dual part of the coordinates), or null
  const int32_t* conn;
  const int32_t* elayer;
  const double* Cl;          // layer stiffness in the material axes, 36 per layer
  const double* Cd;          // its derivative per layer (dual part), or null
  const double* ang;         // ply angle per layer (degrees)
  const double* u;           // displacement (3 per node)
  const double* lam;         // adjoint (3 per node), or null
  const uint8_t* region;     // objective elements, or null (no objective)
  const uint8_t* fixed;      // clamped DOFs
};

struct SensSmem {
  double dNr[27][20][3];
  double X[20][3], Xd[20][3], U[20][3], L[20][3];
  double red[27][61];
  double part[2][64];
};

// One 64-lane work-group per element, lane q < 27 at Gauss point q.  Outputs per element:
// s[e] = derivative part of lambda_e^T K_e u_e, jv[e] = J_e (value), jd[e] = derivative
// part of J_e; with grad != null (value mode) grad[60 e + 3 a + i] receives dJ_e/du of
// element node a, component i (k_grad_gather sums them per node).
template <class R>
__global__ void __launch_bounds__(64) k_sens(SensArgs A, int64_t n_elems, double* s,
                                             double* jv, double* jd, double* grad) {
  extern __shared__ double smem_raw[];
  SensSmem& sm = *reinterpret_cast<SensSmem*>(smem_raw);
  const int t = threadIdx.x;
  for (int idx = t; idx < 27 * 20; idx += 64) {
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
  for (int64_t e = blockIdx.x; e < n_elems; e += gridDim.x) {
    __syncthreads();
    if (t < 60) {
      const int a = t / 3, i = t % 3;
      const int64_t nd = A.conn[20 * e + a];
      sm.X[a][i] = node_coord(A.xyz, nd, i, A.P, e, a);
      sm.Xd[a][i] = A.xd ? A.xd[3 * nd + i] : 0.0;
      sm.U[a][i] = A.u[3 * nd + i];
      sm.L[a][i] = A.lam ? A.lam[3 * nd + i] : 0.0;
    }
    __syncthreads();
    const int layer = A.elayer[e];
    const bool obj = A.region && A.region[e];
    double en_d = 0.0, jq_v = 0.0, jq_d = 0.0;
    if (t < 27) {
      const int q = t;
      R J[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) J[i][j] = mk<R>(0.0, 0.0);
      for (int a = 0; a < 20; ++a)
        for (int i = 0; i < 3; ++i) {
          const R x = mk<R>(sm.X[a][i], sm.Xd[a][i]);
          for (int j = 0; j < 3; ++j) J[i][j] += x * sm.dNr[q][a][j];
        }
      const R det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                    J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                    J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      R Ji[3][3];                                // Ji[j][i] = dxi_j / dx_i
      Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
      Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
      Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
      // material axes: local frame (e1 along dx/dxi, e2 from dx/deta, e3 = e1 x e2), the
      // fibre rotated by the ply angle about e3
      R e1[3] = {J[0][0], J[1][0], J[2][0]}, t2[3] = {J[0][1], J[1][1], J[2][1]};
      const R n1 = dsqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
      for (int i = 0; i < 3; ++i) e1[i] = e1[i] / n1;
      const R pr = t2[0] * e1[0] + t2[1] * e1[1] + t2[2] * e1[2];
      R e2[3] = {t2[0] - pr * e1[0], t2[1] - pr * e1[1], t2[2] - pr * e1[2]};
      const R n2 = dsqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
      for (int i = 0; i < 3; ++i) e2[i] = e2[i] / n2;
      const R e3[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
      const double an = A.ang[layer] * (M_PI / 180.0), ca = cos(an), sa = sin(an);
      R Q[3][3];
      for (int i = 0; i < 3; ++i) {
        Q[0][i] = ca * e1[i] + sa * e2[i];
        Q[1][i] = -sa * e1[i] + ca * e2[i];
        Q[2][i] = e3[i];
      }
      // displacement and adjoint gradients (gu[i][j] = du_i / dx_j)
      R gu[3][3], gl[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gu[i][j] = gl[i][j] = mk<R>(0.0, 0.0);
      for (int a = 0; a < 20; ++a) {
        R gN[3];
        for (int j = 0; j < 3; ++j)
          gN[j] = sm.dNr[q][a][0] * Ji[0][j] + sm.dNr[q][a][1] * Ji[1][j] +
                  sm.dNr[q][a][2] * Ji[2][j];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            gu[i][j] += sm.U[a][i] * gN[j];
            gl[i][j] += sm.L[a][i] * gN[j];
          }
      }
      // engineering strains in the material axes: eps' = Q sym(grad) Q^T
      R vu[6], vl[6];
      {
        R Eu[3][3], El[3][3], Tu[3][3], Tl[3][3];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            Eu[i][j] = 0.5 * (gu[i][j] + gu[j][i]);
            El[i][j] = 0.5 * (gl[i][j] + gl[j][i]);
          }
        for (int i = 0; i < 3; ++i)
          for (int l = 0; l < 3; ++l) {
            Tu[i][l] = Q[i][0] * Eu[0][l] + Q[i][1] * Eu[1][l] + Q[i][2] * Eu[2][l];
            Tl[i][l] = Q[i][0] * El[0][l] + Q[i][1] * El[1][l] + Q[i][2] * El[2][l];
          }
        const int vi[6] = {0, 1, 2, 1, 0, 0}, vj[6] = {0, 1, 2, 2, 2, 1};
        for (int K = 0; K < 6; ++K) {
          const int i = vi[K], j = vj[K];
          const R su = Tu[i][0] * Q[j][0] + Tu[i][1] * Q[j][1] + Tu[i][2] * Q[j][2];
          const R sl = Tl[i][0] * Q[j][0] + Tl[i][1] * Q[j][1] + Tl[i][2] * Q[j][2];
          vu[K] = K < 3 ? su : 2.0 * su;
          vl[K] = K < 3 ? sl : 2.0 * sl;
        }
      }
      const double* Cv = A.Cl + 36 * layer;
      const double* Cdv = A.Cd ? A.Cd + 36 * layer : nullptr;
      R sig[6];
      for (int I = 0; I < 6; ++I) {
        R acc = mk<R>(0.0, 0.0);
        for (int K = 0; K < 6; ++K)
          acc += mk<R>(Cv[6 * I + K], Cdv ? Cdv[6 * I + K] : 0.0) * vu[K];
        sig[I] = acc;
      }
      double xq, wq, yq, wy, zq, wz;
      gauss3(q % 3, &xq, &wq);
      gauss3((q / 3) % 3, &yq, &wy);
      gauss3(q / 9, &zq, &wz);
      const R wdet = det * (wq * wy * wz);
      R en = mk<R>(0.0, 0.0);
      for (int K = 0; K < 6; ++K) en += vl[K] * sig[K];
      en_d = der(en * wdet);
      if (obj) {
        const R jq = sig[2] * sig[2] * wdet;
        jq_v = val(jq);
        jq_d = der(jq);
      }
      if (grad && obj) {
        // dJ_q/du_a = 2 sigma'_3 wdet tau grad N_a, tau = Q^T tau' Q, tau' the tensor form
        // of the third stiffness row (value mode: R = double)
        const double kap = 2.0 * val(sig[2]) * val(wdet);
        double tp[3][3];
        tp[0][0] = Cv[12]; tp[1][1] = Cv[13]; tp[2][2] = Cv[14];
        tp[1][2] = tp[2][1] = Cv[15];
        tp[0][2] = tp[2][0] = Cv[16];
        tp[0][1] = tp[1][0] = Cv[17];
        double tau[3][3];
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) {
            double acc = 0.0;
            for (int i = 0; i < 3; ++i)
              for (int j = 0; j < 3; ++j) acc += val(Q[i][k]) * tp[i][j] * val(Q[j][l]);
            tau[k][l] = kap * acc;
          }
        for (int a = 0; a < 20; ++a) {
          double gN[3];
          for (int j = 0; j < 3; ++j)
            gN[j] = sm.dNr[q][a][0] * val(Ji[0][j]) + sm.dNr[q][a][1] * val(Ji[1][j]) +
                    sm.dNr[q][a][2] * val(Ji[2][j]);
          for (int k = 0; k < 3; ++k)
            sm.red[q][3 * a + k] = tau[k][0] * gN[0] + tau[k][1] * gN[1] + tau[k][2] * gN[2];
        }
      }
    }
    // per-element sums over the Gauss points (fixed order)
    sm.part[0][t] = en_d;
    sm.part[1][t] = jq_v;
    if (t < 27) sm.red[t][60] = jq_d;
    __syncthreads();
    if (t == 0) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      for (int q = 0; q < 27; ++q) {
        a0 += sm.part[0][q];
        a1 += sm.part[1][q];
        a2 += sm.red[q][60];
      }
      if (s) s[e] = a0;
      if (jv) jv[e] = a1;
      if (jd) jd[e] = a2;
    }
    if (grad && t < 60) {
      double acc = 0.0;
      if (obj)
        for (int q = 0; q < 27; ++q) acc += sm.red[q][t];
      grad[60 * e + t] = acc;
    }
  }
}

// dJ/du at every node from the per-element parts ge [60 n_elems] of k_sens: the node's
// elements in ascending order (fixed summation order, no atomics); zero on clamped DOFs
__global__ void k_grad_gather(int64_t n_nodes, const int32_t* ne_ptr, const int32_t* ne_idx,
                              const int32_t* conn, const double* ge, const uint8_t* fixed,
                              double* grad) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= n_nodes) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int32_t k = ne_ptr[n]; k < ne_ptr[n + 1]; ++k) {
    const int64_t e = ne_idx[k];
    int a = 0;
    while (a < 19 && conn[20 * e + a] != (int32_t)n) ++a;
    a0 += ge[60 * e + 3 * a];
    a1 += ge[60 * e + 3 * a + 1];
    a2 += ge[60 * e + 3 * a + 2];
  }
  grad[3 * n] = fixed[3 * n] ? 0.0 : a0;
  grad[3 * n + 1] = fixed[3 * n + 1] ? 0.0 : a1;
  grad[3 * n + 2] = fixed[3 * n + 2] ? 0.0 : a2;
}

// lambda^T df/dp of the face loads: the consistent load of a face (3x3 Gauss rule, traction
// t = t0 + k zeta_c n_out with zeta_c = (x - c) . d the through-thickness coordinate)
// evaluated in dual numbers along dX/dp: the face's normal and area element move with the
// nodes, zeta_c belongs to the laminate and does not; one thread per (face, element node)
__global__ void __launch_bounds__(64) k_face_dload(Periodic P, int64_t n_faces, const int32_t* fe,
                                                  const int32_t* fid,
                             const double* xyz, const double* xd, const int32_t* conn,
                             gx_traction tr, const uint8_t* fixed, const double* lam,
                             double* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_faces * 20) return;
  const int64_t e = fe[idx / 20];
  const int na = (int)(idx % 20);
  const int face = fid[idx / 20];
  const int ax = face / 2;
  const double sgn = (face & 1) ? 1.0 : -1.0;
  Dual fl[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int qb = 0; qb < 3; ++qb)
    for (int qc = 0; qc < 3; ++qc) {
      double pb, wb, pc, wc;
      gauss3(qb, &pb, &wb);
      gauss3(qc, &pc, &wc);
      const double p0 = ax == 0 ? sgn : (ax == 1 ? pc : pb);
      const double p1 = ax == 1 ? sgn : (ax == 2 ? pc : pb);
      const double p2 = ax == 2 ? sgn : (ax == 0 ? pc : pb);
      Dual x[3] = {{0, 0}, {0, 0}, {0, 0}}, tb[3] = {{0, 0}, {0, 0}, {0, 0}},
           tc[3] = {{0, 0}, {0, 0}, {0, 0}};
      double Na = 0.0;
      for (int a = 0; a < 20; ++a) {
        double N, d[3];
        shape_one(a, p0, p1, p2, &N, d);
        const double db = ax == 0 ? d[1] : (ax == 1 ? d[2] : d[0]);
        const double dc = ax == 0 ? d[2] : (ax == 1 ? d[0] : d[1]);
        const int64_t nd = conn[20 * e + a];
        for (int i = 0; i < 3; ++i) {
          const Dual X = {node_coord(xyz, nd, i, P, e, a), xd[3 * nd + i]};
          x[i] += N * X;
          tb[i] += db * X;
          tc[i] += dc * X;
        }
        if (a == na) Na = N;
      }
      const Dual nv[3] = {tb[1] * tc[2] - tb[2] * tc[1], tb[2] * tc[0] - tb[0] * tc[2],
                          tb[0] * tc[1] - tb[1] * tc[0]};
      const Dual dA = dsqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      // the linear part of the traction is a function of the through-thickness coordinate
      // (the load is defined on the laminate, and the wrinkle moves the end face with it):
      // its value comes from the current geometry, it has no derivative in p
      double lin = 0.0;
      for (int i = 0; i < 3; ++i) lin += (x[i].v - tr.c[i]) * tr.d[i];
      lin *= tr.k;
      const Dual w = dA * (wb * wc * Na);
      for (int i = 0; i < 3; ++i)
        fl[i] += (Dual{tr.t0[i], 0.0} + (lin * sgn) * nv[i] / dA) * w;
    }
  const int64_t d = 3 * (int64_t)conn[20 * e + na];
  double r = 0.0;
  for (int i = 0; i < 3; ++i)
    if (!fixed[d + i]) r += lam[d + i] * fl[i].d;
  out[idx] = r;
}

// dC/dE11 per layer: -C (dS/dE11) C for an orthotropic layer (dS11 = -1/E1^2,
// dS12 = nu12/E1^2, dS13 = nu13/E1^2), C / E for an isotropic one (C linear in E)
__global__ void k_layer_dC(int n_layers, const double* eng, const double* C, double* dC) {
  const int L = blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= n_layers) return;
  const double* p = eng + 9 * L;
  const double* c = C + 36 * L;
  double* o = dC + 36 * L;
  if (!(p[3] > 0)) {
    for (int i = 0; i < 36; ++i) o[i] = c[i] / p[0];
    return;
  }
  const double E1 = p[0], n12 = p[6], n13 = p[7];
  double dS[3][3] = {{-1.0 / (E1 * E1), n12 / (E1 * E1), n13 / (E1 * E1)},
                     {n12 / (E1 * E1), 0.0, 0.0},
                     {n13 / (E1 * E1), 0.0, 0.0}};
  // only the normal block of S depends on E1: dC = -C[:, 0:3] dS C[0:3, :]
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc += c[6 * i + k] * dS[k][l] * c[6 * l + j];
      o[6 * i + j] = -acc;
    }
}

// fixed-order sums: out[k] = sum of v[e] over the elements with key[e] == k (key null: k = 0)
__global__ void k_keyed_sum(int64_t n, const double* v, const int32_t* key, int n_keys,
                            double* out) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256)
    if (!key || key[i] == k) acc += v[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && k < n_keys) out[k] = red[0];
}

// sum of v[0..n) in a fixed order, through the one-value device buffer o
static double dev_sum_into(const double* v, int64_t n, double* o, hipStream_t st) {
  hipLaunchKernelGGL(k_keyed_sum, dim3(1), dim3(256), 0, st, n, v, (const int32_t*)nullptr, 1,
                     o);
  GX_HIP(hipGetLastError());
  double h = 0.0;
  to_host(&h, o, 1, st);
  return h;
}

static double dev_sum(const double* v, int64_t n, hipStream_t st) {
  DevBuf<double> o(1);
  return dev_sum_into(v, n, o.p, st);
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static SensArgs sens_args(gx_ctx* c, const double* u, const double* lam, const double* xd,
                          const double* Cd, const uint8_t* region) {
  return SensArgs{periodic_of(c), c->xyz.p, xd, c->conn.p, c->elayer.p, c->Cl.p, Cd, c->ang.p, u,
                  lam, region, c->fixed.p};
}

static unsigned sens_grid(int64_t E) { return (unsigned)std::min<int64_t>(E, 256 * 64); }

static void check_objective_laminate(gx_ctx* c, const gx_laminate* lam) {
  int64_t nn = 0, ne = 0;
  laminate_sizes(lam, &nn, &ne);
  GX_REQUIRE(nn == c->n_nodes && ne == c->n_elems, "laminate does not match the assembled mesh");
}

// J and (grad != null) dJ/du [3 n_nodes], with the caller's buffers: region [n_elems] (the
// element mask), jv [n_elems] (J per element), sum [1] and, with grad, ge [60 n_elems]
static double objective_into(gx_ctx* c, const gx_laminate* lam, int32_t region_kind,
                             const double* u, uint8_t* region, double* jv, double* sum,
                             double* ge, double* grad) {
  hipStream_t st = c->stream;
  const int64_t E = c->n_elems;
  if (region_kind == 0) {
    hipLaunchKernelGGL(k_fill_u8, dim3(nblocks(E, 256)), dim3(256), 0, st, region, E,
                       (uint8_t)1);
    GX_HIP(hipGetLastError());
  } else {
    laminate_region(lam, region, st);
  }
  hipLaunchKernelGGL(k_sens<double>, dim3(sens_grid(E)), dim3(64), sizeof(SensSmem), st,
                     sens_args(c, u, nullptr, nullptr, nullptr, region), E, (double*)nullptr,
                     jv, (double*)nullptr, ge);
  GX_HIP(hipGetLastError());
  if (grad) {
    hipLaunchKernelGGL(k_grad_gather, dim3(nblocks(c->n_nodes, 256)), dim3(256), 0, st,
                       c->n_nodes, c->ne_ptr.p, c->ne_idx.p, c->conn.p, ge, c->fixed.p, grad);
    GX_HIP(hipGetLastError());
  }
  return dev_sum_into(jv, E, sum, st);
}

static double objective(gx_ctx* c, const gx_laminate* lam, int32_t region_kind, const double* u,
                        DevBuf<uint8_t>& region, double* grad) {
  check_objective_laminate(c, lam);
  const int64_t E = c->n_elems;
  region.alloc(E);
  DevBuf<double> jv(E), sum(1), ge(grad ? 60 * E : 0);
  return objective_into(c, lam, region_kind, u, region.p, jv.p, sum.p, ge.p, grad);
}

// ---- scratch of the allocation-free objective (gx_objective_noalloc)
// One array per device, held until the process ends.  In host code the name `scratch` only
// stands for the symbol: its device address comes from hipGetSymbolAddress (per device, in
// noalloc_scratch_init) and only that address is ever passed to kernels or copies.
constexpr size_t NOALLOC_BYTES = GX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;           // device address per device (null: unset)

// Resolve the scratch array's address on `device`, which must be current (gx_create).
void noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  GX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Error(GX_EHIP, "hipGetSymbolAddress returned a null scratch address");
  g_scratch_ptr[device] = p;
}

static unsigned char* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device >= (int)g_scratch_ptr.size() || !g_scratch_ptr[device])
    throw Error(GX_ESTATE, "the scratch array of this device was not set up");
  return static_cast<unsigned char*>(g_scratch_ptr[device]);
}

}  // namespace gx

using namespace gx;

extern "C" {

gx_status gx_objective(gx_ctx* c, const gx_laminate* lam, int32_t region, const double* u,
                       double* J_out) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "matrix not assembled");
  if (c->matrix_only) throw Error(GX_ESTATE, "needs an assembled mesh, not a loaded matrix");
  GX_REQUIRE(lam && u && J_out && (region == 0 || region == 1), "bad objective arguments");
  DevBuf<uint8_t> mask;
  *J_out = objective(c, lam, region, u, mask, nullptr);
  GX_API_END(c)
}

gx_status gx_objective_noalloc(gx_ctx* c, const gx_laminate* lam, int32_t region,
                               const double* u, double* J_out) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "matrix not assembled");
  if (c->matrix_only) throw Error(GX_ESTATE, "needs an assembled mesh, not a loaded matrix");
  GX_REQUIRE(lam && u && J_out && (region == 0 || region == 1), "bad objective arguments");
  check_objective_laminate(c, lam);
  // layout: the sum at 0, J per element at 256, the region mask after it
  const int64_t E = c->n_elems;
  const size_t need = 256 + 8 * (size_t)E + (size_t)E;
  if (need > NOALLOC_BYTES)
    throw Error(GX_EINVAL, "mesh too large for the allocation-free objective: " +
                               std::to_string(need) + " bytes of scratch needed, " +
                               std::to_string(NOALLOC_BYTES) + " available");
  unsigned char* base = noalloc_scratch(c->device);
  double* sum = reinterpret_cast<double*>(base);
  double* jv = reinterpret_cast<double*>(base + 256);
  uint8_t* mask = base + 256 + 8 * (size_t)E;
  *J_out = objective_into(c, lam, region, u, mask, jv, sum, nullptr, nullptr);
  GX_API_END(c)
}

gx_status gx_adjoint(gx_ctx* c, const gx_laminate* lam, int32_t region, const double* u,
                     double rtol, int32_t maxit, double* J_out, double* dJdp,
                     int32_t* iters_out) {
  GX_API_BEGIN(c)
  if (!c->setup_done) throw Error(GX_ESTATE, "gx_geneo_setup has not been called");
  GX_REQUIRE(lam && u && dJdp && (region == 0 || region == 1) && rtol > 0 && maxit > 0,
             "bad adjoint arguments");
  GX_REQUIRE(lam->n_layers <= c->n_layers, "the laminate has more layers than the ply stack");
  hipStream_t st = c->stream;
  const int64_t n = 3 * c->n_nodes, E = c->n_elems;
  const int nl = c->n_layers;
  // objective and its gradient dJ/du (zero on the clamped DOFs)
  DevBuf<uint8_t> mask;
  DevBuf<double> g(n), lamv(n);
  zero(g, st);
  zero(lamv, st);
  const double J = objective(c, lam, region, u, mask, g.p);
  if (J_out) *J_out = J;
  // adjoint solve K lambda = dJ/du with the same preconditioner
  int32_t it = 0;
  double rr = 0.0;
  const gx_status ps = gx_pcg_solve(c, g.p, lamv.p, rtol, maxit, &it, &rr, nullptr);
  if (ps != GX_OK && ps != GX_ENOCONV) throw Error(ps, c->err);
  if (iters_out) *iters_out = it;
  DevBuf<double> s(E), jd(E), xd(n), fd(std::max<int64_t>(c->n_faces * 20, 1));
  // shape parameters: wrinkle amplitude and wavelength
  for (int p = 0; p < 2; ++p) {
    laminate_velocity(lam, p, xd.p, st);
    hipLaunchKernelGGL(k_sens<Dual>, dim3(sens_grid(E)), dim3(64), sizeof(SensSmem), st,
                       sens_args(c, u, lamv.p, xd.p, nullptr, mask.p), E, s.p,
                       (double*)nullptr, jd.p, (double*)nullptr);
    GX_HIP(hipGetLastError());
    const double dK = dev_sum(s.p, E, st), dJ = dev_sum(jd.p, E, st);
    double df = 0.0;
    if (c->n_faces > 0) {
      hipLaunchKernelGGL(k_face_dload, dim3(nblocks(c->n_faces * 20, 64)), dim3(64), 0, st,
                         periodic_of(c), c->n_faces, c->face_e.p, c->face_id.p, c->xyz.p, xd.p, c->conn.p,
                         c->traction, c->fixed.p, lamv.p, fd.p);
      GX_HIP(hipGetLastError());
      df = dev_sum(fd.p, c->n_faces * 20, st);
    }
    dJdp[p] = dJ - (dK - df);
  }
  // E11 of every layer (the loads do not depend on the moduli)
  DevBuf<double> eng(9 * nl), dC(36 * nl), dK(nl), dJ(nl);
  to_dev(eng.p, c->eng.data(), 9 * nl, st);
  hipLaunchKernelGGL(k_layer_dC, dim3(nblocks(nl, 64)), dim3(64), 0, st, nl, eng.p, c->Cl.p,
                     dC.p);
  hipLaunchKernelGGL(k_sens<Dual>, dim3(sens_grid(E)), dim3(64), sizeof(SensSmem), st,
                     sens_args(c, u, lamv.p, nullptr, dC.p, mask.p), E, s.p, (double*)nullptr,
                     jd.p, (double*)nullptr);
  hipLaunchKernelGGL(k_keyed_sum, dim3(nl), dim3(256), 0, st, E, s.p, c->elayer.p, nl, dK.p);
  hipLaunchKernelGGL(k_keyed_sum, dim3(nl), dim3(256), 0, st, E, jd.p, c->elayer.p, nl, dJ.p);
  GX_HIP(hipGetLastError());
  std::vector<double> hK(nl), hJ(nl);
  to_host(hK.data(), dK.p, nl, st);
  to_host(hJ.data(), dJ.p, nl, st);
  for (int L = 0; L < nl; ++L) dJdp[2 + L] = hJ[L] - hK[L];
  if (ps == GX_ENOCONV)                            // outputs are filled from the last iterate
    throw Error(GX_ENOCONV, "adjoint solve did not reach rtol in maxit iterations");
  GX_API_END(c)
}

}  // extern "C"
