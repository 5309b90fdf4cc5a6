// placeholder, replaced by the Krylov-Schur driver
#include "ctx.hpp"
extern "C" int lind_eigs(lind_ctx*, int, double, double, double, void*, void*, lind_info*) { return LIND_EINVAL; }
extern "C" int lind_steady_grad(lind_ctx*, const void*, double, double*, void*, void*, void*, lind_info*) { return LIND_EINVAL; }
