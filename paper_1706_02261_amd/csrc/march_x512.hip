// Persistent march kernels for rows of length 512 (all column lengths).
#include "march_kernels.hpp"

namespace bpm {
BPM_MARCH_INSTANTIATE(512)
}  // namespace bpm
