// Kernel tables of 2D quadrilateral meshes: the gas (Euler + passive species)
// and drift-diffusion models on four-vertex cells.
#include "vcx_internal.h"

using namespace vcx;

const KernelTable* vcx::pick_table_quad(const vcx_physics& ph) {
  if (ph.model == VCX_MODEL_GAS) {
    switch (ph.nspecies) {
      case 0: return pick_flux_prec<0, 2, 0, 4>(ph.flux, ph.precision);
      case 2: return pick_flux_prec<0, 2, 2, 4>(ph.flux, ph.precision);
      case 9: return pick_flux_prec<0, 2, 9, 4>(ph.flux, ph.precision);
      default: return nullptr;
    }
  }
  if (ph.model == VCX_MODEL_DRIFT_DIFFUSION) {
    switch (ph.nspecies) {
      case 1: return pick_flux_prec<1, 2, 1, 4>(0, ph.precision);
      case 2: return pick_flux_prec<1, 2, 2, 4>(0, ph.precision);
      default: return nullptr;
    }
  }
  return nullptr;
}
