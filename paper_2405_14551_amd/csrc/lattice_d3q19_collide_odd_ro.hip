// Collision-pass instantiations: D3Q19, odd streaming, read-once true.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D3Q19, STREAM_ODD, true)
