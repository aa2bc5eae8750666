// batched.hip -- many independent SVDs of uneven sizes (placeholder: the
// per-matrix plain path; replaced by the persistent kernel).
#include <hip/hip_runtime.h>

#include "../../include/jsvd.h"
#include "kernels.hpp"

extern "C" int jsvd_gesvj_batched(int count, const int *m, const int *n, const int *is_complex,
                                  double *const *G_re, double *const *G_im, const size_t *ldg,
                                  double *const *V_re, double *const *V_im, const size_t *ldv,
                                  double *const *sv_e, double *const *sv_f, int max_sweeps, int *sweeps,
                                  int *status, unsigned flags, void *stream)
{
    if (count < 0 || (count > 0 && (!m || !n || !G_re || !ldg || !V_re || !ldv || !sv_e || !sv_f || !status)))
        return JSVD_EINVAL;
    int rc_all = JSVD_OK;
    for (int i = 0; i < count; ++i) {
        const int cplx = is_complex ? is_complex[i] : 0;
        int sw = 0;
        const int rc = jsvd_gesvj(m[i], n[i], G_re[i], cplx ? G_im[i] : nullptr, ldg[i], V_re[i],
                                  cplx ? V_im[i] : nullptr, ldv[i], sv_e[i], sv_f[i], nullptr, max_sweeps, &sw,
                                  flags, stream);
        status[i] = rc;
        if (sweeps) sweeps[i] = sw;
        if (rc < 0 && rc_all == JSVD_OK) rc_all = rc;
    }
    return rc_all;
}
