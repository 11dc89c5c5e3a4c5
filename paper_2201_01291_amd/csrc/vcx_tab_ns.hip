// Kernel tables of the multi-species Navier-Stokes model: every (dimension, species, flux,
// precision) instantiation of its tile kernels and launchers.
#include "vcx_internal.h"

using namespace vcx;

const KernelTable* vcx::pick_table_ns(int nd, const vcx_physics& ph) {
  if (ph.flux != VCX_FLUX_HLLC) return nullptr;
  switch (ph.nspecies) {
    case 2: return nd == 2 ? pick_flux_prec<2, 2, 2>(0, ph.precision) : pick_flux_prec<2, 3, 2>(0, ph.precision);
    case 9: return nd == 2 ? pick_flux_prec<2, 2, 9>(0, ph.precision) : pick_flux_prec<2, 3, 9>(0, ph.precision);
    default: return nullptr;
  }
}
