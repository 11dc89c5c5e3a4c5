// Kernel tables of the 3D gas (Euler + passive species) model: every (dimension, species, flux,
// precision) instantiation of its tile kernels and launchers.
#include "vcx_internal.h"

using namespace vcx;

const KernelTable* vcx::pick_table_gas3(const vcx_physics& ph) {
  switch (ph.nspecies) {
    case 0: return pick_flux_prec<0, 3, 0>(ph.flux, ph.precision);
    case 2: return pick_flux_prec<0, 3, 2>(ph.flux, ph.precision);
    case 9: return pick_flux_prec<0, 3, 9>(ph.flux, ph.precision);
    default: return nullptr;
  }
}
