// Trace / Fisher building blocks (trace.hip).
#pragma once
#include "hm_factor.h"

namespace hm {

hm_status dots(Model* m, const double* const* A, int na, const double* const* B, int nb, long len, double* out,
               double* partial);
// out[i nb + j] = sum over leaves of tr(A_i[L] B_j[L]) (leaf-major nl x nl blocks)
hm_status dots_leafT(Model* m, const double* const* A, int na, const double* const* B, int nb, double* out,
                     double* partial);
hm_status sum_scalar(Model* m, const double* x, long len, int diag_nl, double* out, double* partial);
hm_status param_prepare(FactorCtx& f, ParamBufs& pb, const double* theta, const double* tF_prefix,
                        const double* GtG);
hm_status scale_sweep(FactorCtx& f, ParamBufs& ps, const ParamBufs& pt, const double* theta);
hm_status tangent_sweep(FactorCtx& f, ParamBufs& pb);
hm_status node_prep(FactorCtx& f);
hm_status node_psi(FactorCtx& f, ParamBufs& pb, double* xtmp);
hm_status node_lam(FactorCtx& f, ParamBufs& pb, double* tbuf, double* dsbuf);
hm_status panel_products(FactorCtx& f, ParamBufs& pb);

}  // namespace hm
