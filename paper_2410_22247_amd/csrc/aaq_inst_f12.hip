// Kernel instantiations for complex64 amplitudes and tiles of 2^12 amplitudes.
#include "aaq_engine.h"

AAQ_INSTANTIATE_UNITS(float, 12, f12)
AAQ_INSTANTIATE_SWEEPS(float, 12, f12)
