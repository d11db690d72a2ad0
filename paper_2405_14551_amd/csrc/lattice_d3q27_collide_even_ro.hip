// Collision-pass instantiations: D3Q27, even streaming, read-once true.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D3Q27, STREAM_EVEN, true)
