// Entry points not implemented yet (return FE_ENOTSUP).
#include "fe_internal.h"

using namespace fe;

namespace fe {
hipError_t launch_nonlocal(const fe_mesh *, const double *, int64_t, double *, int64_t, int64_t, double, double *,
                           hipStream_t) {
    return hipErrorNotSupported;
}
size_t nonlocal_work_doubles(const fe_mesh *, int64_t) { return 0; }
}  // namespace fe

extern "C" {
fe_status fe_set_nonlocal(fe_mesh *, int32_t, const double *, const double *, double, double, hipStream_t) {
    return fail(FE_ENOTSUP, "nonlocal term not implemented");
}
}
