// Whole-mesh launchers at P = 4.
#define SHP_P 4
#include "shp_k_mixed_p.inc"
