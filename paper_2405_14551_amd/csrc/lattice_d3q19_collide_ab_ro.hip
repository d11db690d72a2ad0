// Collision-pass instantiations: D3Q19, ab streaming, read-once true; read-once ensemble launches.
#include "collide_launch.hpp"

LB_INSTANTIATE_COLLIDE(D3Q19, STREAM_AB, true)
LB_INSTANTIATE_ENSEMBLE_RO(D3Q19)
