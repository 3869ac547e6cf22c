// Kernels of the prism shape.
#define SHP_SHAPE PRISM
#define SHP_FN(name) name##prism
#include "shp_k_shape.inc"
