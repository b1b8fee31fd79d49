// fdtd_launch.hpp -- host-side launcher declarations (kernels live in the .hip files).
#pragma once
#include "fdtd_dev.hpp"

// psi pre-pass of x and z over axes d0 .. d0 + nd - 1 (y and fused shots skipped); max_count =
// largest slab of those axes
void fdtd_launch_psi(int stor, const DevShot *d_shots, int nshots, long max_count, int iu, int ext, int d0, int nd,
                     hipStream_t st);
// psi_y pre-pass along y lines; max_lines = largest nx * Nz of the shots
void fdtd_launch_psi_y(int stor, const DevShot *d_shots, int nshots, long max_lines, int iu, int ext, hipStream_t st);
void fdtd_launch_naive(int stor, const DevShot *d_shots, int shot, int nx, int Ny, int Nz, const Roles &R,
                       const int *stepc, hipStream_t st);
// z-march of the points outside the bands: cols x points per lane (1: tiles of
// 64 x 8 ry points, 2: 128 x 8 ry)
void fdtd_launch_zmarch(int stor, const DevShot *d_shots, const WorkItem *work, int nwork, int ry, int cols,
                        const Roles &R, int zchunk, const int *stepc, hipStream_t st);
// band points (tiles of every box kind in one list; ty = BAND_TY or BAND_TY_TALL rows per tile)
void fdtd_launch_band(int stor, const DevShot *d_shots, const BandItem *work, int nwork, const Roles &R, int zchunk,
                      const int *stepc, int ty, hipStream_t st);
void fdtd_launch_record(int stor, const DevShot *d_shots, int nshots, const Roles &R, int *stepc, hipStream_t st);
// temporal blocking: args points to a host TBArgs (kernels_tblock.hip); K = 2 or 4
void fdtd_launch_tblock(const DevShot *d_shots, const WorkItem *work, int nwork, int K, const void *args, int zchunk,
                        const int *stepc, hipStream_t st);
int fdtd_tblock_core(int K, int axis);
struct TBArgsHost {
    int blo[3], bhi[3];
    int L[6];
    const int *rec_zs;
    const int *rec_ix;
};

void fdtd_launch_fill_zero(void *p, size_t bytes, hipStream_t st);
void fdtd_launch_vel_to_m(const float *v, float *m, int nx, int ny, int nz, int P, int S, double dt2,
                          unsigned int *vmax_bits, unsigned int *bad, hipStream_t st);
void fdtd_launch_get_field(int stor, const void *u, float *dst, int nx, int ny, int nz, int P, int S, float inv,
                           hipStream_t st);
void fdtd_launch_set_field(int stor, void *u, const float *src, int nx, int ny, int nz, int P, int S, float sc,
                           hipStream_t st);
void fdtd_launch_finite(int stor, const void *u, int nx, int ny, int nz, int P, int S, unsigned int *bad,
                        hipStream_t st);
void fdtd_launch_get_prev(int stor, const void *u, const void *d, float *dst, int nx, int ny, int nz, int P, int S,
                          float inv, hipStream_t st);
void fdtd_launch_set_prev(int stor, const void *u, void *d, const float *src, int nx, int ny, int nz, int P, int S,
                          float sc, hipStream_t st);
// strided box copies (CopyJob list); max_rows = most rows (ey * ez) of a job
void fdtd_launch_copy_jobs(const void *jobs, int njobs, long max_rows, hipStream_t st);
void fdtd_launch_set_int(int *p, int v, hipStream_t st);
void fdtd_launch_stream_probe(const float *a, const float *b, const float *c, float *o, size_t n4, int blocks,
                              int unroll, hipStream_t st);
