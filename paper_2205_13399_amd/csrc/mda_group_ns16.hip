// mda_group_ns16.hip -- the workgroup form built for 16 register slots per lane.
#define MDA_TILE 16
#include "mda_group_tile.h"
