// Collision-pass instantiations: D2Q9, even streaming, read-once false.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D2Q9, STREAM_EVEN, false)
