// mda_generic_k3.hip -- the K-objective kernels for K = 3 (every slot count).
#define MDA_GK 3
#include "mda_generic_tile.h"
