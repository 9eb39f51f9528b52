// Persistent march kernels for rows of length 32 (all column lengths).
#include "march_kernels.hpp"

namespace bpm {
BPM_MARCH_INSTANTIATE(32)
}  // namespace bpm
