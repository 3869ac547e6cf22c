// Whole-mesh launchers at P = 2.
#define SHP_P 2
#include "shp_k_mixed_p.inc"
