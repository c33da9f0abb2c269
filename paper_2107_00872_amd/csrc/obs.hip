// Observables (Sec. 3.6, 4.2), S^-_q (Alg. 11) and the dynamical structure
// factor (Sec. 3.9).
#include <hip/hip_runtime.h>

#include "qs3_impl.h"

using namespace qs3;

extern "C" {
int qs3_sz(qs3_sector *, const void *, double *, void *) { set_error("not built yet"); return QS3_EINVAL; }
int qs3_sisj(qs3_sector *, const void *, int, const int32_t *, const int32_t *, double *, double *, void *) { set_error("not built yet"); return QS3_EINVAL; }
int qs3_sq(qs3_sector *, const void *, int, const double *, double *, double *, double *, void *) { set_error("not built yet"); return QS3_EINVAL; }
int qs3_smq(qs3_sector *, const void *, qs3_sector *, const int32_t *, void *, void *) { set_error("not built yet"); return QS3_EINVAL; }
int qs3_dsf(qs3_sector *, const void *, double, int, const int32_t *, const qs3_dsf_opts *, int, const double *, double *, double *, double *, double *, void *) { set_error("not built yet"); return QS3_EINVAL; }
}
