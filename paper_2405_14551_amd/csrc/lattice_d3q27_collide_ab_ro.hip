// Collision-pass instantiations: D3Q27, ab streaming, read-once true; read-once ensemble launches.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D3Q27, STREAM_AB, true)
LB_INSTANTIATE_ENSEMBLE_RO(D3Q27)
