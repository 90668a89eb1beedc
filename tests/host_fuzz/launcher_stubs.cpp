// Stand-ins for the kernel launchers (p1e_kernels.hip) so that the host setup code links into a
// CPU-only program for the sanitizer build; every one reports a HIP error and none is reached
// by the fuzz, which never binds a mesh.
#include "p1e_internal.h"
namespace p1e {
int run_energy(p1e_mesh *, const double *, int, double *, int32_t *, hipStream_t) { return P1E_EHIP; }
int run_grad_exact(p1e_mesh *, const double *, int, double *, double *, int32_t *, hipStream_t) { return P1E_EHIP; }
int run_grad_fd(p1e_mesh *, const double *, double, int, double *, int32_t *, hipStream_t) { return P1E_EHIP; }
int run_energy_forces(p1e_mesh *, const double *, int, double *, int32_t *, hipStream_t) { return P1E_EHIP; }
int run_scale(p1e_mesh *, const double *, double *, hipStream_t) { return P1E_EHIP; }
int run_scale_inplace(p1e_mesh *, const double *, double *, hipStream_t) { return P1E_EHIP; }
int run_grad_exact_static(p1e_mesh *, const double *, int, double *, double *, int32_t *, hipStream_t) { return P1E_EHIP; }
uint64_t static_scratch_need(const p1e_mesh *) { return 0; }
}
