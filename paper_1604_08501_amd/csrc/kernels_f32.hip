// Single-order kernels, float instantiation.
#define SEM_REAL float
#include "kernels.inc"
