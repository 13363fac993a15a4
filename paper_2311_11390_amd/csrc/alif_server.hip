// Serving: continuous batching of independent single-layer simulations.
// (implementation follows; entry points report ALIF_EUNSUPPORTED until then)
#include <hip/hip_runtime.h>

#include "../../include/blockalif.h"
#include "alif_kernels.h"

extern "C" {
int alif_server_create(size_t, int32_t, int32_t, alif_server **) {
    return alif::set_error(ALIF_EUNSUPPORTED, "serving not built");
}
int alif_request_footprint(const alif_request *, size_t *) {
    return alif::set_error(ALIF_EUNSUPPORTED, "serving not built");
}
int alif_submit(alif_server *, const alif_request *, uint64_t *) {
    return alif::set_error(ALIF_EUNSUPPORTED, "serving not built");
}
int alif_poll(alif_server *, uint64_t, alif_result *) {
    return alif::set_error(ALIF_EUNSUPPORTED, "serving not built");
}
int alif_server_destroy(alif_server *) { return ALIF_OK; }
}
