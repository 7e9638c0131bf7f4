// Batched exponentials: see expm_sparse_batched in expm.h.
#include "../../include/expm.h"

extern "C" int expm_sparse_batched(expm_plan_t p, int count, const expm_csr_cview *H,
                                   const double *eps, expm_csr *E) {
    (void)p;
    (void)count;
    (void)H;
    (void)eps;
    (void)E;
    return EXPM_ENOTIMPL;
}
