// Launchers of the libtbsma kernels (host side).
#pragma once

#include "tbsma_device.hpp"

namespace tbsma {

void launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                     hipStream_t s);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
void launch_set_step(int64_t *p, int64_t v, hipStream_t s);
void launch_quantise(const Dev &S, hipStream_t s);
// Work lists of the step from the rebuild and pruning flags (all replicas
// rebuild when S.all); read by the cell, list-build and pruning kernels.
void launch_worklist(const Dev &S, hipStream_t s);
void launch_cells(const Dev &S, hipStream_t s);
// List build of the replicas that rebuild (all when S.all); in mixed
// precision also the lane-ordered rows of those and of the replicas whose
// lists are pruned this step.
void launch_nlist(const Dev &S, bool mixed, double rl, hipStream_t s);
void launch_block_map(const Dev &S, hipStream_t s);
void launch_list_stats(const Dev &S, bool mixed, hipStream_t s);
void launch_forces(const Dev &S, bool mixed, const PotF &PF, const PotD &PD,
                   void *fx, void *fy, void *fz, void *eat, double *g,
                   hipStream_t s);
// Both mixed pair passes of a step-loop step, the force pass ending with the
// second half kick and kinetic sums (replaces launch_integrate_b).
void launch_forces_kick(const Dev &S, const DevMD &M, const PotF &PF,
                        void *fx, void *fy, void *fz, void *eat,
                        hipStream_t s);
void launch_force_pass(const Dev &S, bool mixed, int pass, const PotF &PF,
                       const PotD &PD, void *fx, void *fy, void *fz, void *eat,
                       double *g, hipStream_t s);
void launch_reduce_forces(const Dev &S, double *re, double *rw,
                          hipStream_t s);
void launch_integrate_a(const Dev &S, const DevMD &M, bool mixed,
                        const void *fx, const void *fy, const void *fz,
                        hipStream_t s);
void launch_integrate_b(const Dev &S, const DevMD &M, bool mixed,
                        const void *fx, const void *fy, const void *fz,
                        hipStream_t s);
void launch_reduce_step(const Dev &S, const DevMD &M, hipStream_t s);
// Start of a step-loop call of n steps: records its first and end step
// (read by the deferred second half kick).
void launch_call_bounds(const Dev &S, const DevMD &M, int64_t n,
                        hipStream_t s);
// Start of a step-loop call: Nose-Hoover and barostat state from the
// current velocities and forces.
void launch_step_begin(const Dev &S, const DevMD &M, bool mixed,
                       const void *fz, hipStream_t s);
void launch_nh_finish(const Dev &S, const DevMD &M, hipStream_t s);
void launch_init(const Dev &S, const DevMD &M, bool mixed, double jitter,
                 hipStream_t s);
// Per-replica dof, constant volume and grip faces from the atoms as they are.
void launch_replica_constants(const Dev &S, double r0, int32_t *dof,
                              double *vol, double *z_lo, double *z_hi,
                              hipStream_t s);
// z0 = z; L0 += 2 s and s, ds/dt = 0 for each replica (baro_s may be NULL).
void launch_rebase(const Dev &S, double *L0, double *baro_s, hipStream_t s);
// Philox words, FP64 normals and FP32 normals (each output may be NULL).
void launch_rng_fill(uint64_t seed, uint32_t rep, uint64_t step,
                     uint32_t stream, int64_t n, uint32_t *w, double *g,
                     float *gf, hipStream_t s);

}  // namespace tbsma
