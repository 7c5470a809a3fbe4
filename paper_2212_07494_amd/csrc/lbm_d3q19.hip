// Kernels of the D3Q19 lattice (see lbm_lattice_impl.h).
#define LBM_LAT D3Q19
#define LBM_OPS ops_d3q19
#include "lbm_lattice_impl.h"
