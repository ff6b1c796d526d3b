// Kernels and launchers of the bf16 storage path.
#include "lbm_engine_impl.h"

namespace lbm {
template struct Engine<bf16_t>;
}  // namespace lbm
