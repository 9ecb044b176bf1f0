// mda_wave64_ns16.hip -- the one-wave kernel with int64 energy differences,
// built for 16 register slots per lane (instances of up to 16 facilities).
#define MDA_TILE 16
#define MDA_F64 1
#include "mda_wave_tile.h"
