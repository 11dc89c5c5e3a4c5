// Kernel tables of the drift-diffusion model: every (dimension, species, flux,
// precision) instantiation of its tile kernels and launchers.
#include "vcx_internal.h"

using namespace vcx;

const KernelTable* vcx::pick_table_dd(int nd, const vcx_physics& ph) {
  switch (ph.nspecies) {
    case 1: return nd == 2 ? pick_flux_prec<1, 2, 1>(0, ph.precision) : pick_flux_prec<1, 3, 1>(0, ph.precision);
    case 2: return nd == 2 ? pick_flux_prec<1, 2, 2>(0, ph.precision) : pick_flux_prec<1, 3, 2>(0, ph.precision);
    default: return nullptr;
  }
}
