// Allocation-free residual (vcx_residual_noalloc in include/vcx.h): the
// residual of a caller-supplied device state, computed by the same kernels as
// vcx_residual, with every intermediate array (reconstructed rows, nodal
// gradients, tile partials, staged field, output in internal order) placed in
// one fixed device array of this library instead of solver buffers.
#include <mutex>

#include "vcx_internal.h"

namespace {

// per device, held until the process ends
constexpr size_t kScratchDoubles = size_t(8) << 20;  // 64 MiB
constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

}  // namespace

// The scratch array.  In host code its name is only a host-side stand-in: the
// device address on each device comes from hipGetSymbolAddress (above).
static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of the scratch array on device `dev`, resolved once per
// device with that device current.
static vcx_status scratch_on(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(VCX_E_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    VCX_HIP(hipGetDevice(&cur));
    if (cur != dev) VCX_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail(VCX_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return VCX_OK;
}

// carve n doubles from the scratch, 256-byte aligned
static double* carve(double* base, size_t& off, size_t n) {
  double* p = base + off;
  off += (std::max<size_t>(n, 1) + 31) / 32 * 32;
  return p;
}

extern "C" size_t vcx_noalloc_scratch_bytes(void) { return sizeof(double) * kScratchDoubles; }

extern "C" vcx_status vcx_residual_noalloc(vcx_mesh mesh, const vcx_physics* phys, const double* U,
                                           const double* E, double dt, double* r) {
  if (!mesh || !phys || !U || !r) return fail(VCX_E_ARG, "NULL argument");
  const vcx_physics& ph = *phys;
  const KernelTable* kt = nullptr;
  VCX_TRY(check_physics(mesh, ph, E, &kt));
  // a host-side solver record pointing into the scratch (no device memory
  // of its own)
  vcx_solver_s s;
  VCX_TRY(configure_solver(&s, mesh, ph, kt));
  const DevMesh& d = mesh->d;
  const size_t nn = (size_t)d.nn, P = (size_t)d.nslots;
  const bool dd = ph.model == VCX_MODEL_DRIFT_DIFFUSION;
  // required doubles, each array rounded up to 256 bytes
  auto rnd = [](size_t n) { return (std::max<size_t>(n, 1) + 31) / 32 * 32; };
  const size_t nws_d = staged_doubles(nn, s.ldws, s.nd, ph.nspecies, g_fp32(&s));
  const size_t need = rnd((size_t)s.nw * nn) + (s.ldws ? rnd(nws_d) : 0) + rnd((size_t)node_row(s.ngf * s.nd) * nn) +
                      rnd((size_t)s.ngf * s.nd * P) + rnd((size_t)s.nvar * P) + rnd((size_t)s.nvar * nn) +
                      (dd ? rnd((size_t)s.nd * nn) : 0) +
                      (ph.closure == 2 && d.nb > 0 ? rnd((size_t)d.nb * s.nvar) : 0);
  if (need > kScratchDoubles)
    return fail(VCX_E_ARG, "mesh too large for the allocation-free residual: needs " +
                               std::to_string(need * sizeof(double)) + " B of scratch, the limit is " +
                               std::to_string(kScratchDoubles * sizeof(double)) + " B");
  double* base = nullptr;
  VCX_TRY(scratch_on(mesh->device, &base));
  size_t off = 0;
  s.W[0] = carve(base, off, (size_t)s.nw * nn);
  if (s.ldws) s.WS[0] = carve(base, off, nws_d);
  s.cur = 0;
  s.G = carve(base, off, (size_t)node_row(s.ngf * s.nd) * nn);
  s.PG = carve(base, off, (size_t)s.ngf * s.nd * P);
  s.PR = carve(base, off, (size_t)s.nvar * P);
  s.rbuf = carve(base, off, (size_t)s.nvar * nn);
  if (dd) s.E = carve(base, off, (size_t)s.nd * nn);
  if (ph.closure == 2 && d.nb > 0) s.cbuf = carve(base, off, (size_t)d.nb * s.nvar);
  if (s.fused && dd && ph.closure && d.nb > 0) s.gout = s.G;
  hipStream_t st = mesh->stream;
  const dim3 nb((unsigned)((nn + 255) / 256)), blk(256);
  // caller order -> internal order: state rows, then the field
  hipLaunchKernelGGL(k_gather_rows, nb, blk, 0, st, d.perm, U, s.W[0], (int)nn, s.nvar);
  if (dd) hipLaunchKernelGGL(k_gather_rows, nb, blk, 0, st, d.perm, E, s.E, (int)nn, s.nd);
  VCX_HIP(hipGetLastError());
  VCX_TRY(kt->aux(&s, s.W[0]));
  // the residual passes of vcx_residual
  const double* Win = s.W[0];
  Finish f = make_finish(&s);
  f.Win = Win;
  f.rout = s.rbuf;
  f.residual_only = 1;
  if (s.fused) {
    FusedCtl fc{nullptr, 0, 0, s.gout};
    VCX_TRY(kt->fused(&s, Win, f, fc, dt));
  } else {
    GradCtl gc{nullptr, 0, 0};
    VCX_TRY(kt->grad(&s, Win, gc, false));
    if (ph.closure == 2) VCX_TRY(kt->closure2(&s, f));
    VCX_TRY(kt->flux(&s, Win, f, dt));
  }
  VCX_TRY(kt->update_shared(&s, f));
  hipLaunchKernelGGL(k_scatter_rows, nb, blk, 0, st, d.perm, (const double*)s.rbuf, r, (int)nn, s.nvar);
  VCX_HIP(hipGetLastError());
  // the scratch is reused by the next call: return only when this one is done
  VCX_HIP(hipStreamSynchronize(st));
  return VCX_OK;
}
