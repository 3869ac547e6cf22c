// Kernels of the pyr shape.
#define SHP_SHAPE PYR
#define SHP_FN(name) name##pyr
#include "shp_k_shape.inc"
