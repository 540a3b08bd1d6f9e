// 20-node serendipity hexahedron: reference nodes, shape functions and the 3-point Gauss
// rule (section 2.1: quadratic serendipity elements with full integration).  Shared by the
// assembly and the sensitivity kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace gx {

// ---------------------------------------------------------------------------------------
// Serendipity shape functions on the reference cube [-1, 1]^3.
static __device__ __constant__ int8_t c_ref[20][3] = {
    {-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {-1, 1, 1},  {1, 1, 1},
    {0, -1, -1},  {0, 1, -1},  {0, -1, 1},  {0, 1, 1},
    {-1, 0, -1},  {1, 0, -1},  {-1, 0, 1},  {1, 0, 1},
    {-1, -1, 0},  {1, -1, 0},  {-1, 1, 0},  {1, 1, 0}};

// value and reference gradient of shape function a at (p0, p1, p2)
static __device__ inline void shape_one(int a, double p0, double p1, double p2, double* N,
                                        double* d) {
  const double r0 = c_ref[a][0], r1 = c_ref[a][1], r2 = c_ref[a][2];
  const double f0 = 1 + p0 * r0, f1 = 1 + p1 * r1, f2 = 1 + p2 * r2;
  if (r0 != 0 && r1 != 0 && r2 != 0) {
    const double g = p0 * r0 + p1 * r1 + p2 * r2 - 2;
    *N = 0.125 * f0 * f1 * f2 * g;
    d[0] = 0.125 * r0 * f1 * f2 * (g + f0);
    d[1] = 0.125 * r1 * f0 * f2 * (g + f1);
    d[2] = 0.125 * r2 * f0 * f1 * (g + f2);
  } else if (r0 == 0) {                          // edge along xi: bubble (1 - xi^2)
    const double b = 1 - p0 * p0;
    *N = 0.25 * b * f1 * f2;
    d[0] = -0.5 * p0 * f1 * f2;
    d[1] = 0.25 * b * r1 * f2;
    d[2] = 0.25 * b * f1 * r2;
  } else if (r1 == 0) {                          // edge along eta
    const double b = 1 - p1 * p1;
    *N = 0.25 * b * f0 * f2;
    d[0] = 0.25 * b * r0 * f2;
    d[1] = -0.5 * p1 * f0 * f2;
    d[2] = 0.25 * b * f0 * r2;
  } else {                                       // edge along zeta
    const double b = 1 - p2 * p2;
    *N = 0.25 * b * f0 * f1;
    d[0] = 0.25 * b * r0 * f1;
    d[1] = 0.25 * b * f0 * r1;
    d[2] = -0.5 * p2 * f0 * f1;
  }
}

// Coordinates of element nodes of a periodic mesh: node a of element e is seen at its
// stored coordinates plus the period when bit a of wrap[e] is set (wrap null: never).
struct Periodic {
  const uint32_t* wrap;
  double p[3];
};

static __device__ inline double node_coord(const double* xyz, int64_t nd, int i,
                                           const Periodic& P, int64_t e, int a) {
  double x = xyz[3 * nd + i];
  if (P.wrap && ((P.wrap[e] >> a) & 1u)) x += P.p[i];
  return x;
}

// the context's description (defined where gx_ctx is complete)
template <class Ctx>
inline Periodic periodic_of(const Ctx* c) {
  Periodic P;
  P.wrap = c->wrap.p;
  for (int i = 0; i < 3; ++i) P.p[i] = c->period[i];
  return P;
}

static __device__ inline void gauss3(int i, double* x, double* w) {
  const double s = 0.7745966692414833770358531;  // sqrt(3/5)
  *x = (i == 0) ? -s : ((i == 1) ? 0.0 : s);
  *w = (i == 1) ? 8.0 / 9.0 : 5.0 / 9.0;
}


}  // namespace gx
