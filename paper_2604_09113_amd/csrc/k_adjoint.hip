// Compliance gradient (A11).  Placeholder entry points; the adjoint
// contraction kernels are added in the same file.
#include "internal.h"

extern "C" lbddc_status lbddc_compliance_gradient(lbddc_ctx*, double*, double*, double*) { return LBDDC_E_UNSUPPORTED; }
extern "C" lbddc_status lbddc_compliance_gradient_device(lbddc_ctx*, double*, double*, double*) { return LBDDC_E_UNSUPPORTED; }
