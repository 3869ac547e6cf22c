// Whole-mesh launchers at P = 10.
#define SHP_P 10
#include "shp_k_mixed_p.inc"
