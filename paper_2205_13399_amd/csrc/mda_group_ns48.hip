// mda_group_ns48.hip -- the workgroup form built for 48 register slots per lane.
#define MDA_TILE 48
#include "mda_group_tile.h"
