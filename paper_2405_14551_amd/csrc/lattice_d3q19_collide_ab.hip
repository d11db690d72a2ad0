// Collision-pass instantiations: D3Q19, ab streaming, read-once false.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D3Q19, STREAM_AB, false)
