// Kernels and launchers of the f16 storage path.
#include "lbm_engine_impl.h"

namespace lbm {
template struct Engine<_Float16>;
}  // namespace lbm
