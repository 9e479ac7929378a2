// stubs.hip -- entry points not built yet.
#include "kmpp_dev.h"
#include "kmpp_impl.h"

namespace kmpp {
size_t batched_workspace(const kmpp_instance*, int) { return 256; }
int batched_prepare(const kmpp_instance*, int, uint64_t, void*, size_t, hipStream_t) { return KMPP_E_UNSUPPORTED; }
int batched_launch(void*, hipStream_t) { return KMPP_E_UNSUPPORTED; }
}  // namespace kmpp
