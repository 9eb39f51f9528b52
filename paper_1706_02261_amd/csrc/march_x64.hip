// Persistent march kernels for rows of length 64 (all column lengths).
#include "march_kernels.hpp"

namespace bpm {
BPM_MARCH_INSTANTIATE(64)
}  // namespace bpm
