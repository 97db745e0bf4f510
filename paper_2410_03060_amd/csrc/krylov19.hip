// Krylov solvers and products for wires of 20 segments (19 rooftop unknowns,
// the discretisation of the paper's own runs, Sec. II-A).
#define CHAFF_KNB 19
#define CHAFF_KNS kr19
#include "krylov_impl.hpp"
