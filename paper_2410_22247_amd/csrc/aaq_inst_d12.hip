// Kernel instantiations for complex128 amplitudes and tiles of 2^12 amplitudes.
#include "aaq_engine.h"

AAQ_INSTANTIATE_UNITS(double, 12, d12)
AAQ_INSTANTIATE_SWEEPS(double, 12, d12)
