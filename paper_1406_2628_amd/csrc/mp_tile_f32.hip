// Per-tile merge kernels for float keys.
#include "mp_tile_impl.h"
MP_TILE_INSTANTIATE(float)
