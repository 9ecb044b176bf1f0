// mda_generic_k1.hip -- the K-objective kernels for K = 1 (every slot count).
#define MDA_GK 1
#define MDA_GX_HOME 1
#include "mda_generic_tile.h"
