// Kernels of the D2Q9 lattice (see lbm_lattice_impl.h).
#define LBM_LAT D2Q9
#define LBM_OPS ops_d2q9
#include "lbm_lattice_impl.h"
