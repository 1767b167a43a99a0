// PSM stream-collide instantiations for double PDF storage.
#include "k_stream_collide.hpp"

#define PSM_T double
#define PSM_LAUNCH_NAME launch_sc_f64
#include "k_sc_launch.inc"
