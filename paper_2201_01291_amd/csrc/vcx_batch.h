// Library-internal interface of batch groups: the solves that one launch per
// kernel advances together.  Used by the C ABI (vcx_solve_batch) and by the
// request scheduler of the serving API.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "vcx.h"
#include "vcx_mesh.h"

namespace vcx {

struct BatchGroup;

// A group enqueues its work on `stream`.  With `graphs`, two consecutive
// batch steps are captured once per membership into a HIP graph and
// replayed; otherwise every kernel is launched directly.
vcx_status batch_create(hipStream_t stream, bool graphs, BatchGroup** out);
void batch_destroy(BatchGroup* g);
size_t batch_size(const BatchGroup* g);

// Replace the members (n >= 0).  Members must be batch-compatible, have a
// state and idle streams.  steps_left[i] >= 0 is each member's remaining
// step budget and t_end[i] its end time (<= 0: none); both are copied.
vcx_status batch_set(BatchGroup* g, vcx_solver* ss, int n, const int* steps_left, const double* t_end);

// Enqueue nsteps batch steps (no host synchronisation).
vcx_status batch_run(BatchGroup* g, int nsteps);

// Commit the pending step of every member, wait for the group's stream and
// update the members' host-side counters (time, steps, buffer parity,
// failure flag).  ended[i] = 1 once member i can make no further progress
// (failed, budget spent or end time reached).
vcx_status batch_sync(BatchGroup* g, std::vector<int>* ended);

// Same model, scheme and kernel instantiation.
bool batch_compatible(vcx_solver a, vcx_solver b);

// Device bytes a solver of this physics on this mesh allocates.
vcx_status solver_footprint(vcx_mesh mesh, const vcx_physics* phys, size_t* bytes);

// Reuse of a solver for a new request: same mesh and byte-identical
// physics; a drift-diffusion solver takes the new request's field.
bool solver_matches(vcx_solver s, vcx_mesh mesh, const vcx_physics* ph);
vcx_status solver_set_field(vcx_solver s, const double* E);

// Small accessors and the thread's error message (vcx_last_error).
vcx_status set_error(vcx_status s, const char* msg);
int mesh_ndim(vcx_mesh m);
int64_t mesh_nnodes(vcx_mesh m);
const HostMesh* mesh_host(vcx_mesh m);        // preprocessed mesh, internal order
bool mesh_axisymmetric(vcx_mesh m);
// cells are simplices (not 2D quadrilaterals)
bool mesh_simplex(vcx_mesh m);
hipStream_t mesh_stream(vcx_mesh m);          // stream of the mesh and its solvers
const int32_t* mesh_perm_device(vcx_mesh m);  // [nn] internal node -> caller node (device)
int solver_failed(vcx_solver s);

}  // namespace vcx
