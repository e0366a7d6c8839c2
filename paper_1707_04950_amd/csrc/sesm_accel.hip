// Shifted-equivalent-source FFT accelerator (Sec. 5): placeholder until the
// accelerated forward map lands; dense mode is the only operator for now.
#include "sesm_impl.h"

int sesm_accel_setup(sesm_ctx* ctx) { return ctx->fail(SESM_EINVAL, "accelerated mode not built yet"); }
int sesm_accel_matvec(sesm_ctx* ctx, const cplx*, cplx*) { return ctx->fail(SESM_EINVAL, "accelerated mode not built yet"); }
void sesm_accel_free(sesm_ctx*) {}
void sesm_accel_info(const sesm_ctx*, sesm_surface_info*) {}
