// PSM stream-collide instantiations for float PDF storage.
#include "k_stream_collide.hpp"

#define PSM_T float
#define PSM_LAUNCH_NAME launch_sc_f32
#include "k_sc_launch.inc"
