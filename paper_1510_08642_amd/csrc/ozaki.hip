// placeholder, replaced by the Ozaki INT8 path
#include "../../include/ddqd.h"
#include "common.hpp"
namespace ddqd {
size_t ozaki_workspace(int64_t, int64_t, int64_t, int64_t, int) { return 0; }
int launch_ozaki(const GemmBatch&, int, void*, size_t, hipStream_t) {
  return set_error(DDQD_E_UNSUPPORTED, "Ozaki base not built yet");
}
int ozaki_default_slices() { return 16; }
}  // namespace ddqd
