// Kernels of the D3Q39 lattice (see lbm_lattice_impl.h).
#define LBM_LAT D3Q39
#define LBM_OPS ops_d3q39
#include "lbm_lattice_impl.h"
