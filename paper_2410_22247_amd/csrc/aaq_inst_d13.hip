// Kernel instantiations for complex128 amplitudes and tiles of 2^13 amplitudes.
#include "aaq_engine.h"

AAQ_INSTANTIATE_UNITS(double, 13, d13)
AAQ_INSTANTIATE_SWEEPS(double, 13, d13)
