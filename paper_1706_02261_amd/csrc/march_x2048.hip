// Persistent march kernels for rows of length 2048 (all column lengths).
#include "march_kernels.hpp"

namespace bpm {
BPM_MARCH_INSTANTIATE(2048)
}  // namespace bpm
