// Persistent march kernels for rows of length 1024 (all column lengths).
#include "march_kernels.hpp"

namespace bpm {
BPM_MARCH_INSTANTIATE(1024)
}  // namespace bpm
