// Whole-mesh launchers at P = 6.
#define SHP_P 6
#include "shp_k_mixed_p.inc"
