// PSM stream-collide instantiations for _Float16 PDF storage.
#include "k_stream_collide.hpp"

#define PSM_T _Float16
#define PSM_LAUNCH_NAME launch_sc_f16
#include "k_sc_launch.inc"
