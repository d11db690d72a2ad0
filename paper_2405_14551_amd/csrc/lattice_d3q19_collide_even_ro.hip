// Collision-pass instantiations: D3Q19, even streaming, read-once true.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D3Q19, STREAM_EVEN, true)
