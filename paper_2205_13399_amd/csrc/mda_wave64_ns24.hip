// mda_wave64_ns24.hip -- the one-wave kernel with int64 energy differences,
// built for 24 register slots per lane (instances of up to 24 facilities).
#define MDA_TILE 24
#define MDA_F64 1
#include "mda_wave_tile.h"
