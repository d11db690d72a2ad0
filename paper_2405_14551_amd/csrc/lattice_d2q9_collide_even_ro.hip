// Collision-pass instantiations: D2Q9, even streaming, read-once true.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D2Q9, STREAM_EVEN, true)
