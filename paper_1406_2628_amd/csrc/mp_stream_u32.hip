// Persistent merge kernels instantiated for uint32_t keys (see mp_stream_impl.h).
#include "mp_stream_impl.h"

MP_STREAM_INSTANTIATE(uint32_t)
