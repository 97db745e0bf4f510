// Krylov solvers and products for wires of 8 segments (7 rooftop unknowns).
#define CHAFF_KNB 7
#define CHAFF_KNS kr7
#include "krylov_impl.hpp"
