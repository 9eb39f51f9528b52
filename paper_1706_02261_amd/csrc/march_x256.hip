// Persistent march kernels for rows of length 256 (all column lengths).
#include "march_kernels.hpp"

namespace bpm {
BPM_MARCH_INSTANTIATE(256)
}  // namespace bpm
