// Through-thickness stresses and the delamination-onset criterion (section 3.3).
//
// The paper assesses the strength of the curved laminate with the quadratic criterion of
// Camanho et al. (Eq. eq-Camanho),
//
//   F = sqrt( (sigma_r^+ / s33)^2 + (tau_rs / s13)^2 + (tau_rl / s13)^2 ),
//
// sigma_r^+ = max(sigma_r, 0), evaluated in the resin interface layers only; failure
// initiates at F = 1, and since the problem is linear the moment at initiation is M / max F.
//
// Stresses are recovered at the 27 Gauss points of every selected element from the
// displacement: the strain of u_e, rotated into the material axes (the geometric frame
// e1 = unit dx/dxi, e2 = dx/deta made orthogonal, e3 = e1 x e2, turned by the ply angle
// about e3, as in the assembly), times the layer stiffness, then turned back by the ply
// angle into the frame (s, l, r) = (e1, e2, e3).  One 64-lane work-group per element, lane q
// at Gauss point q; the element's maximum goes to a per-element slot, and one work-group
// reduces those in a fixed order (ties go to the lower element, then the lower point), so
// the result is the same on every run.
#include <cmath>

#include "element.h"
#include "gx_internal.h"

namespace gx {

struct FailSmem {
  double X[20][3];
  double U[20][3];
  double F[64];
  double S[64][6];
};

__global__ void __launch_bounds__(64) k_failure(Periodic P, int64_t n_elems, const double* xyz,
                                                const int32_t* conn, const int32_t* elayer,
                                                const double* Cl, const double* ang,
                                                const uint8_t* sel, const double* u,
                                                double s33, double s13, double* Fq,
                                                double* Fe, int32_t* qe, double* Se) {
  __shared__ FailSmem sm;
  const int t = threadIdx.x;
  for (int64_t e = blockIdx.x; e < n_elems; e += gridDim.x) {
    const int layer = elayer[e];
    if (!sel[layer]) {                           // uniform per work-group
      if (t < 27 && Fq) Fq[27 * e + t] = 0.0;
      if (t == 0) {
        Fe[e] = 0.0;
        qe[e] = 0;
      }
      if (t < 6) Se[6 * e + t] = 0.0;
      continue;
    }
    __syncthreads();
    if (t < 60) {
      const int a = t / 3, i = t % 3;
      const int64_t nd = conn[20 * e + a];
      sm.X[a][i] = node_coord(xyz, nd, i, P, e, a);
      sm.U[a][i] = u[3 * nd + i];
    }
    __syncthreads();
    double F = -1.0, loc[6] = {0, 0, 0, 0, 0, 0};
    if (t < 27) {
      double p0, p1, p2, w;
      gauss3(t % 3, &p0, &w);
      gauss3((t / 3) % 3, &p1, &w);
      gauss3(t / 9, &p2, &w);
      double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int a = 0; a < 20; ++a) {
        double N, d[3];
        shape_one(a, p0, p1, p2, &N, d);
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) J[i][j] += sm.X[a][i] * d[j];
      }
      const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      const double id = 1.0 / det;
      double Ji[3][3];                           // Ji[j][i] = dxi_j / dx_i
      Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
      Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
      Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
      // displacement gradient H[i][j] = du_i / dx_j
      double H[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int a = 0; a < 20; ++a) {
        double N, d[3];
        shape_one(a, p0, p1, p2, &N, d);
        double g[3];
        for (int i = 0; i < 3; ++i) g[i] = d[0] * Ji[0][i] + d[1] * Ji[1][i] + d[2] * Ji[2][i];
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) H[i][j] += sm.U[a][i] * g[j];
      }
      // geometric frame (rows of E) and material axes (rows of Q)
      double E[3][3];
      {
        double n1 = sqrt(J[0][0] * J[0][0] + J[1][0] * J[1][0] + J[2][0] * J[2][0]);
        for (int i = 0; i < 3; ++i) E[0][i] = J[i][0] / n1;
        const double pr = J[0][1] * E[0][0] + J[1][1] * E[0][1] + J[2][1] * E[0][2];
        for (int i = 0; i < 3; ++i) E[1][i] = J[i][1] - pr * E[0][i];
        const double n2 = sqrt(E[1][0] * E[1][0] + E[1][1] * E[1][1] + E[1][2] * E[1][2]);
        for (int i = 0; i < 3; ++i) E[1][i] /= n2;
        E[2][0] = E[0][1] * E[1][2] - E[0][2] * E[1][1];
        E[2][1] = E[0][2] * E[1][0] - E[0][0] * E[1][2];
        E[2][2] = E[0][0] * E[1][1] - E[0][1] * E[1][0];
      }
      const double an = ang[layer] * (M_PI / 180.0), ca = cos(an), sa = sin(an);
      double Q[3][3];
      for (int i = 0; i < 3; ++i) {
        Q[0][i] = ca * E[0][i] + sa * E[1][i];
        Q[1][i] = -sa * E[0][i] + ca * E[1][i];
        Q[2][i] = E[2][i];
      }
      // strain in the material axes, eps' = Q sym(H) Q^T, engineering Voigt vector
      double em[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double acc = 0.0;
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) acc += Q[a][i] * 0.5 * (H[i][j] + H[j][i]) * Q[b][j];
          em[a][b] = acc;
        }
      const double ev[6] = {em[0][0], em[1][1], em[2][2], 2.0 * em[1][2], 2.0 * em[0][2],
                            2.0 * em[0][1]};
      const double* C = Cl + 36 * layer;
      double sv[6];
      for (int I = 0; I < 6; ++I) {
        double acc = 0.0;
        for (int K = 0; K < 6; ++K) acc += C[6 * I + K] * ev[K];
        sv[I] = acc;
      }
      // back to the frame (s, l, r): sigma_geo = Rp sigma' Rp^T, Rp the rotation by the ply
      // angle about e3 (Rp[a][m] = e_a . q_m)
      const double Sm[3][3] = {{sv[0], sv[5], sv[4]}, {sv[5], sv[1], sv[3]}, {sv[4], sv[3], sv[2]}};
      const double Rp[3][3] = {{ca, -sa, 0.0}, {sa, ca, 0.0}, {0.0, 0.0, 1.0}};
      double Sg[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double acc = 0.0;
          for (int m = 0; m < 3; ++m)
            for (int k = 0; k < 3; ++k) acc += Rp[a][m] * Sm[m][k] * Rp[b][k];
          Sg[a][b] = acc;
        }
      loc[0] = Sg[0][0];
      loc[1] = Sg[1][1];
      loc[2] = Sg[2][2];
      loc[3] = Sg[1][2];
      loc[4] = Sg[0][2];
      loc[5] = Sg[0][1];
      const double sr = loc[2] > 0.0 ? loc[2] / s33 : 0.0;
      const double trs = loc[4] / s13, trl = loc[3] / s13;
      F = sqrt(sr * sr + trs * trs + trl * trl);
      if (Fq) Fq[27 * e + t] = F;
    }
    sm.F[t] = F;
    for (int k = 0; k < 6; ++k) sm.S[t][k] = loc[k];
    __syncthreads();
    if (t == 0) {
      int best = 0;
      for (int q = 1; q < 27; ++q)
        if (sm.F[q] > sm.F[best]) best = q;
      Fe[e] = sm.F[best];
      qe[e] = best;
      for (int k = 0; k < 6; ++k) Se[6 * e + k] = sm.S[best][k];
    }
  }
}

// The largest F over all elements (ties: the lower element index) by one work-group in a
// fixed order: each thread scans a strided set of elements, then a tree over the threads.
__global__ void __launch_bounds__(256) k_failure_max(int64_t n_elems, const double* Fe,
                                                     int64_t* best_e) {
  __shared__ double v[256];
  __shared__ int64_t ix[256];
  const int t = threadIdx.x;
  double bv = -1.0;
  int64_t bi = -1;
  for (int64_t e = t; e < n_elems; e += 256)
    if (Fe[e] > bv) {
      bv = Fe[e];
      bi = e;
    }
  v[t] = bv;
  ix[t] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      const double ov = v[t + w];
      const int64_t oi = ix[t + w];
      if (ov > v[t] || (ov == v[t] && oi >= 0 && (ix[t] < 0 || oi < ix[t]))) {
        v[t] = ov;
        ix[t] = oi;
      }
    }
    __syncthreads();
  }
  if (t == 0) *best_e = ix[0];
}

}  // namespace gx

using namespace gx;

extern "C" gx_status gx_failure(gx_ctx* c, const double* u, const int32_t* layer_mask,
                                double s33, double s13, double* F_gauss, double* F_elem,
                                gx_failure_result* out) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "matrix not assembled");
  if (c->matrix_only) throw Error(GX_ESTATE, "needs an assembled mesh, not a loaded matrix");
  GX_REQUIRE(u && out && s33 > 0 && s13 > 0, "bad failure-criterion arguments");
  hipStream_t st = c->stream;
  const int64_t E = c->n_elems;
  const int nl = c->n_layers;
  std::vector<uint8_t> hs(nl);
  int nsel = 0;
  for (int k = 0; k < nl; ++k) {
    // default: the isotropic layers (G12 <= 0 marks an isotropic entry of the ply stack)
    hs[k] = layer_mask ? (layer_mask[k] != 0) : !(c->eng[9 * k + 3] > 0);
    nsel += hs[k];
  }
  GX_REQUIRE(nsel > 0, "no layer selected for the failure criterion");
  DevBuf<uint8_t> sel(nl);
  to_dev(sel.p, hs.data(), nl, st);
  DevBuf<double> fe, se;
  DevBuf<int32_t> qe(E);
  DevBuf<int64_t> be(1);
  double* Fe = F_elem;
  if (!Fe) {
    fe.alloc(E);
    Fe = fe.p;
  }
  se.alloc(6 * E);
  hipLaunchKernelGGL(k_failure, dim3((unsigned)std::min<int64_t>(E, 256 * 64)), dim3(64), 0, st,
                     periodic_of(c), E, c->xyz.p, c->conn.p, c->elayer.p, c->Cl.p, c->ang.p, sel.p, u, s33, s13,
                     F_gauss, Fe, qe.p, se.p);
  hipLaunchKernelGGL(k_failure_max, dim3(1), dim3(256), 0, st, E, Fe, be.p);
  GX_HIP(hipGetLastError());
  int64_t e = -1;
  to_host(&e, be.p, 1, st);
  GX_REQUIRE(e >= 0 && e < E, "no element of the selected layers");
  int32_t q = 0;
  int32_t layer = 0;
  to_host(&out->F_max, Fe + e, 1, st);
  to_host(&q, qe.p + e, 1, st);
  to_host(&layer, c->elayer.p + e, 1, st);
  to_host(out->stress, se.p + 6 * e, 6, st);
  out->elem = e;
  out->gauss = q;
  out->layer = layer;
  GX_API_END(c)
}
