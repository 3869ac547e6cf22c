// Kernels of the tet shape.
#define SHP_SHAPE TET
#define SHP_FN(name) name##tet
#include "shp_k_shape.inc"
