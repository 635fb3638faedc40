// Kernel instantiations for complex128 amplitudes and tiles of 2^10 amplitudes.
#include "aaq_engine.h"

AAQ_INSTANTIATE_UNITS(double, 10, d10)
