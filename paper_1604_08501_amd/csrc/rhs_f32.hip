// Whole-rate (volume + surface) kernel, float instantiation.
#define SEM_REAL float
#include "rhs.inc"
