// hisq_eigensolve: thick-restart Lanczos with a Chebyshev filter (in progress).
#include "hisq_internal.h"

using namespace hisq;

extern "C" hisq_status hisq_eigensolve(hisq_gauge g, double two_m, int n_ev,
                                       const hisq_eig_params *params, void *evecs_dev,
                                       double *evals_host, hisq_eig_stats *stats_host,
                                       void *stream) {
    (void)g; (void)two_m; (void)n_ev; (void)params; (void)evecs_dev; (void)evals_host;
    (void)stats_host; (void)stream;
    return fail(HISQ_ERR_UNSUPPORTED, "hisq_eigensolve is not implemented yet");
}
