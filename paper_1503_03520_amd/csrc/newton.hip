// Second-order path and FP64 polish (placeholders until the PCG kernels land).
#include "common.hpp"

l1ls_status polish_fp64(const l1ls_instance*, double, double*, hipStream_t, int* r, int64_t* p) {
    *r = 0;
    *p = 0;
    return L1LS_E_UNSUPPORTED;
}

extern "C" l1ls_status l1ls_solve_cg_newton(const l1ls_instance* I, const l1ls_solve_opts* o, double* x,
                                            l1ls_report* rep) {
    if (!I || !o || !x) return L1LS_E_ARG;
    (void)rep;
    return L1LS_E_UNSUPPORTED;
}
