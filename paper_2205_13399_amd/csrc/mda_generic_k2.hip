// mda_generic_k2.hip -- the K-objective kernels for K = 2 (every slot count).
#define MDA_GK 2
#include "mda_generic_tile.h"
