// Kernels and launchers of the f32 storage path.
#include "lbm_engine_impl.h"

namespace lbm {
template struct Engine<float>;
}  // namespace lbm
