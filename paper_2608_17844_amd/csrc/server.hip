// Serving loop: placeholder until the continuous-batching server is built.
#include "runtime.h"

extern "C" {
mbt_status mbt_server_create(mbt_ctx*, int32_t, size_t, mbt_server**) { return MBT_EINVAL; }
mbt_status mbt_server_submit(mbt_server*, const mbt_request*, uint64_t*) { return MBT_EINVAL; }
mbt_status mbt_server_wait(mbt_server*, uint64_t, int32_t, mbt_result**) { return MBT_EINVAL; }
void mbt_result_free(mbt_result*) {}
double mbt_server_clock(const mbt_server*) { return 0; }
void mbt_server_destroy(mbt_server*) {}
}
