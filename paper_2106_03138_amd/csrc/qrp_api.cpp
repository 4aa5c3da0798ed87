// QRP entry points (Algorithm 2 of the paper).  Temporary form: the QRDM
// machinery with a single pivot per step (k_DM = 1), which is Algorithm 2 step
// for step with a rank-1 compact-WY trailing update.
#include <hip/hip_runtime.h>

#include "../../include/qrdm.h"

extern "C" int qrp_factor_ex(double *A, int64_t m, int64_t n, int64_t lda, const qrdm_params *pin, int32_t nb,
                             double *tau_house, int32_t *perm, int64_t *rank, qrdm_stats *stats, void *stream) {
    (void)nb;
    qrdm_params p;
    if (pin) p = *pin; else qrdm_default_params(&p);
    p.tau = 1.0;
    p.delta = 0.0;
    p.kmax = 1;
    return qrdm_factor_ex(A, m, n, lda, &p, tau_house, perm, rank, stats, nullptr, 0, nullptr, stream);
}
