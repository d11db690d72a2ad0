// Collision-pass instantiations: D3Q27, odd streaming, read-once true.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D3Q27, STREAM_ODD, true)
