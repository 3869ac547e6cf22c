// Whole-mesh launchers at P = 9.
#define SHP_P 9
#include "shp_k_mixed_p.inc"
