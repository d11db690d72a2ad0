// Collision-pass instantiations: D2Q9, odd streaming, read-once true.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D2Q9, STREAM_ODD, true)
