// Kernels of the D3Q27 lattice (see lbm_lattice_impl.h).
#define LBM_LAT D3Q27
#define LBM_OPS ops_d3q27
#include "lbm_lattice_impl.h"
