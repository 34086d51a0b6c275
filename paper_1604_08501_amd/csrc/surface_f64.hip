// Surface-term kernel, double instantiation.
#define SEM_REAL double
#include "surface.inc"
