// The integrator variants beside the stored-scalar one, for the ODE and
// root-finding interior methods: a field derived from the maps at every sample
// (the parametrisation quality of Eq. (paramQuality), von Mises of a
// displacement spline, Eq. (vonMises)), and the instrumented integrator that
// records the pixel accuracy (Eq. (deltaP), covering order).  The block is
// read from global memory (the displacement shares its indexing).
#include "ivr_integrate.h"

namespace ivr {

template <int P, bool RAT, int METHOD, int FIELD, bool DIAG>
static hipError_t launch_field_m(bool fp64, const Model &m, const ViewRec *views, int n_views, void *segs,
                                 const IntegrateArgs &a, unsigned long long *ctr, int n_cu, const LaunchCfg &lc,
                                 hipStream_t st) {
    if (fp64)
        return launch_integrate_t<P, RAT, double, false, METHOD, FIELD, DIAG>(m, views, n_views, segs, a, ctr, n_cu,
                                                                              lc, st);
    return launch_integrate_t<P, RAT, float, false, METHOD, FIELD, DIAG>(m, views, n_views, segs, a, ctr, n_cu, lc,
                                                                         st);
}

template <int P, bool RAT, int METHOD>
static hipError_t launch_field_mm(bool fp64, int field, bool diag, const Model &m, const ViewRec *views,
                                  int n_views, void *segs, const IntegrateArgs &a, unsigned long long *ctr, int n_cu,
                                  const LaunchCfg &lc, hipStream_t st) {
    if (diag) return launch_field_m<P, RAT, METHOD, 0, true>(fp64, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    if (field == IVR_FIELD_PARAM_QUALITY)
        return launch_field_m<P, RAT, METHOD, 1, false>(fp64, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    return launch_field_m<P, RAT, METHOD, 2, false>(fp64, m, views, n_views, segs, a, ctr, n_cu, lc, st);
}

template <int P, bool RAT>
static hipError_t launch_field_pr(bool fp64, int method, int field, bool diag, const Model &m, const ViewRec *views,
                                  int n_views, void *segs, const IntegrateArgs &a, unsigned long long *ctr, int n_cu,
                                  const LaunchCfg &lc, hipStream_t st) {
    if (method == IVR_INTERIOR_RF)
        return launch_field_mm<P, RAT, kRootFinding>(fp64, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc,
                                                     st);
    return launch_field_mm<P, RAT, kOde>(fp64, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc, st);
}

hipError_t launch_integrate_field(bool fp64, int method, int field, bool diag, int klass, const Model &m,
                                  const ViewRec *views, int n_views, void *segs, const IntegrateArgs &a,
                                  unsigned long long *ctr, int n_cu, const LaunchCfg &lc, hipStream_t st) {
    if (method != IVR_INTERIOR_ODE && method != IVR_INTERIOR_RF) return hipErrorInvalidValue;
    if (diag ? field != IVR_FIELD_SCALAR : (field != IVR_FIELD_PARAM_QUALITY && field != IVR_FIELD_VON_MISES))
        return hipErrorInvalidValue;
    switch (klass) {
    case 0: return launch_field_pr<1, false>(fp64, method, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 1: return launch_field_pr<1, true>(fp64, method, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 2: return launch_field_pr<2, false>(fp64, method, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 3: return launch_field_pr<2, true>(fp64, method, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 4: return launch_field_pr<3, false>(fp64, method, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    case 5: return launch_field_pr<3, true>(fp64, method, field, diag, m, views, n_views, segs, a, ctr, n_cu, lc, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ivr
