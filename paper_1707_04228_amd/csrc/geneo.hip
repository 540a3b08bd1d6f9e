// GenEO coarse space and the setup entry point of the two-level Schwarz preconditioner.
#include <cmath>

#include "gx_internal.h"

using namespace gx;

extern "C" {

gx_status gx_geneo_setup(gx_ctx* c, const gx_geneo_opts* o, int32_t* nev_out,
                         int64_t* n0_out) {
  GX_API_BEGIN(c)
  if (!c->assembled) throw Error(GX_ESTATE, "gx_assemble has not been called");
  GX_REQUIRE(o && o->elem_part, "null options");
  GX_REQUIRE(o->n_sub >= 1 && o->n_sub <= 4096, "n_sub out of range");
  GX_REQUIRE(o->overlap >= 1 && o->overlap <= 16, "overlap must be in [1, 16]");
  GX_REQUIRE(o->precision == GX_FP64 || o->precision == GX_MIXED, "bad precision");
  c->setup_done = false;
  c->sw = Schwarz();
  Timer t1(c->stream);
  dd_build(c, o->elem_part, o->n_sub, o->overlap);
  c->phase_ms[1] = t1.ms();
  Timer t2(c->stream);
  interior_factors(c, o->precision);
  c->phase_ms[2] = t2.ms();
  c->phase_ms[3] = c->phase_ms[4] = 0;
  c->sw.two_level = o->coarse != 0;
  if (c->sw.two_level) geneo_coarse(c, o);
  if (nev_out)
    for (int j = 0; j < o->n_sub; ++j) nev_out[j] = c->sw.two_level ? c->sw.nev[j] : 0;
  if (n0_out) *n0_out = c->sw.two_level ? c->sw.n0 : 0;
  c->setup_done = true;
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

gx_status gx_geneo_eigenvalues(gx_ctx* c, int32_t j, double* lam) {
  GX_API_BEGIN(c)
  if (!c->setup_done || !c->sw.two_level) throw Error(GX_ESTATE, "no coarse space");
  GX_REQUIRE(j >= 0 && j < c->sw.n_sub && lam, "bad subdomain index");
  for (size_t k = 0; k < c->sw.lam[j].size(); ++k) lam[k] = c->sw.lam[j][k];
  GX_API_END(c)
}

}  // extern "C"

namespace gx {
void geneo_coarse(gx_ctx* c, const gx_geneo_opts* o) {
  (void)o;
  throw Error(GX_EINVAL, "coarse space not available in this build");
}
}  // namespace gx
