// Per-tile merge kernels for int32_t keys.
#include "mp_tile_impl.h"
MP_TILE_INSTANTIATE(int32_t)
