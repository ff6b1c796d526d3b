// Kernels and launchers of the f64 storage path.
#include "lbm_engine_impl.h"

namespace lbm {
template struct Engine<double>;
}  // namespace lbm
