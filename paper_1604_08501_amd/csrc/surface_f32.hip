// Surface-term kernel, float instantiation.
#define SEM_REAL float
#include "surface.inc"
