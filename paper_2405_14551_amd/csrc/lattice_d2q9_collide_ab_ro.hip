// Collision-pass instantiations: D2Q9, ab streaming, read-once true; read-once ensemble launches.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D2Q9, STREAM_AB, true)
LB_INSTANTIATE_ENSEMBLE_RO(D2Q9)
