// Collision-pass instantiations: D2Q9, ab streaming, read-once true.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D2Q9, STREAM_AB, true)
