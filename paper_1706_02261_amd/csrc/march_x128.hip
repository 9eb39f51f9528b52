// Persistent march kernels for rows of length 128 (all column lengths).
#include "march_kernels.hpp"

namespace bpm {
BPM_MARCH_INSTANTIATE(128)
}  // namespace bpm
