// Host-side launch entry points of the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "pic_dev.hpp"

namespace pic {

// persistent grid sizes (workgroups), multiples of 8 (one share per XCD)
int grid_particles(int dims, int prec, int ncu);
int grid_generic(int ncu);

// one step, split in launches (all read their run set from the batch table)
void launch_sort_chain(int dims, int prec, const BatchTable* bt, int nruns, int grid, hipStream_t s);
void launch_particles(int dims, int prec, int pusher, const BatchTable* bt, int grid, hipStream_t s);
// ant_plane: transverse points of the largest run with a laser antenna (0: none)
// the low-pass filter of the deposited current, before the E update (k_filter.hip)
void launch_filter(int dims, int prec, const BatchTable* bt, int grid, int filter_stages, hipStream_t s);
void launch_fields(int dims, int prec, const BatchTable* bt, int grid, int filter_stages, long long ant_plane,
                   hipStream_t s);
// laser antenna sources: phase 0 adds -dt M^n to B^{n+1/2}, phase 1 -dt J^{n+1/2} to E^{n+1}
void launch_antenna(int prec, const BatchTable* bt, long long max_plane, int phase, int grid, hipStream_t s);
void launch_advance(const BatchTable* bt, int nruns, hipStream_t s);
// laboratory-frame stations of every run of the table (before the advance);
// max_items: station points of the largest station set in the table
void launch_stations(int prec, const BatchTable* bt, long long max_items, int grid, hipStream_t s);

// initialisation (one run)
void launch_init_fields(int dims, int prec, const RunDev* rd, long long npts, hipStream_t s);

// diagnostics (one run)
void launch_cont_pre(int dims, int prec, const RunDev* rd, long long npts, long long cap, hipStream_t s);
void launch_rho(int dims, int prec, const RunDev* rd, double* rho, long long npts, long long cap,
                int use_snap, hipStream_t s);
void launch_cont_post(int dims, int prec, const RunDev* rd, long long npts, long long cap, hipStream_t s);
void launch_gauss(int prec, const RunDev* rd, long long npts, int mode, const double* rhoG, hipStream_t s);
// the current filter's stages applied to a node scalar rho (ping-pong t0/t1);
// returns the array holding the result (rho itself when stages = 0)
const double* launch_filter_nodes(int dims, const RunDev* rd, long long npts, int stages, const double* rho,
                                  double* t0, double* t1, hipStream_t s);
void launch_diag(int dims, int prec, const RunDev* rd, long long npts, long long cap, unsigned what,
                 hipStream_t s);
// B[dst] = B[src] + coef curl E[fbuf]; src/dst < 0 select fbuf / fbuf^1
void launch_bshift(int prec, const RunDev* rd, long long npts, int src, int dst, double coef,
                   hipStream_t s);

// pusher microbenchmark
void launch_copy_bench(const void* src, void* dst, long long n16, hipStream_t s);
void launch_stream_bench(int mode, const void* src, void* dst, long long n16, hipStream_t s);
// this device's batch table of pic_step_batch_noalloc (file-scope device array)
hipError_t batch_scratch(BatchTable** out);
void launch_push_bench(int prec, int pusher, long long n, double dt, const double B[3], void* Ex,
                       void* u, int* cell, void* off, hipStream_t s);

}  // namespace pic
