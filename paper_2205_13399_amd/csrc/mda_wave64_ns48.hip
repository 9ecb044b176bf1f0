// mda_wave64_ns48.hip -- the one-wave kernel with int64 energy differences,
// built for 48 register slots per lane (instances of up to 48 facilities).
#define MDA_TILE 48
#define MDA_F64 1
#include "mda_wave_tile.h"
