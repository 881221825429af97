// Batched persistent launch (placeholder until the persistent kernel lands).
#include "qsv_internal.h"

extern "C" qsv_status qsv_batch_run(qsv_ctx ctx, int nb, const int* nq, const int64_t* gate_off,
                                    const qsv_gate* g, const double* params, int64_t nparams,
                                    const int64_t* term_off, const uint64_t* qmasks,
                                    const double* w, int dtype, double* out, int flags) {
    (void)nb; (void)nq; (void)gate_off; (void)g; (void)params; (void)nparams; (void)term_off;
    (void)qmasks; (void)w; (void)dtype; (void)out; (void)flags;
    if (!ctx) return QSV_ERR_ARG;
    ctx->last_error = "qsv_batch_run: not available in this build";
    return QSV_ERR_ARG;
}
