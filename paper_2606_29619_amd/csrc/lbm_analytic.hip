// lbm_analytic.hip -- the solver passes that read analytic porosity derivatives (lbm_params
// grad_eps / hess_eps, Sec. 3.5), instantiated apart from the differenced ones so that the two
// halves of the library compile in parallel.
#include "lbm_launch.hpp"

namespace lbmh {

template <typename F>
void dispatch_analytic(const lbm_solver *h, F &fn) {
    dispatch_cfg<true>(h, fn);
}

template void dispatch_analytic<MomentsPass>(const lbm_solver *, MomentsPass &);
template void dispatch_analytic<VcorrectPass>(const lbm_solver *, VcorrectPass &);
template void dispatch_analytic<CollidePass>(const lbm_solver *, CollidePass &);
template void dispatch_analytic<PicardPass>(const lbm_solver *, PicardPass &);
template void dispatch_analytic<FusedPass>(const lbm_solver *, FusedPass &);
template void dispatch_analytic<InitPass>(const lbm_solver *, InitPass &);
template void dispatch_analytic<BcRecordsPass>(const lbm_solver *, BcRecordsPass &);
template void dispatch_analytic<BcRebuildPass>(const lbm_solver *, BcRebuildPass &);

}  // namespace lbmh
