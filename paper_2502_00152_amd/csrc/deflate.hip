// hisq_deflate: x0 = V diag(1/(eps + (2m)^2)) V^H b (in progress).
#include "hisq_internal.h"

using namespace hisq;

extern "C" hisq_status hisq_deflate(hisq_gauge g, int n_ev, const void *evecs_dev,
                                    const double *evals_host, double two_m, const void *b_e_dev,
                                    void *x0_e_dev, int nrhs, void *stream) {
    (void)g; (void)n_ev; (void)evecs_dev; (void)evals_host; (void)two_m; (void)b_e_dev;
    (void)x0_e_dev; (void)nrhs; (void)stream;
    return fail(HISQ_ERR_UNSUPPORTED, "hisq_deflate is not implemented yet");
}
