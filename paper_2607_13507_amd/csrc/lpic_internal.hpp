// Internal interface between the C ABI (lpic_api.hip) and the kernels (lpic_kernels.hip).
#pragma once

#include "lpic_device.hpp"

namespace lpic {

constexpr int SORT_BLOCK = 2048;   // particles per workgroup of the sort kernels

void launch_yee(const Tables& T, int prec, int dim, int nblocks, int which, double frac,
                int zero_j, hipStream_t st);
void launch_gather_push(const Tables& T, int prec, int dim, int nblocks, void* old,
                        hipStream_t st);
void launch_deposit(const Tables& T, int prec, int dim, int nblocks, const void* old,
                    int with_rho, hipStream_t st);
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t st);
void launch_sort(const Tables& T, int prec, int dim, int nblocks, int32_t* counts,
                 int32_t* offsets, int32_t* cursor, int32_t* mult, int nbins, hipStream_t st);
void launch_swap_segments(SegDesc* segs, int nsegs, hipStream_t st);
void launch_build_chunks(const Tables& T, const int32_t* offsets, int nbins, int chunk,
                         Chunk* out, int32_t* nchunks, hipStream_t st);
void launch_fused(const Tables& T, int prec, int dim, int nblocks, size_t smem,
                  const Chunk* chunks, const int32_t* nchunks, int with_rho, double* kinetic,
                  int ke_to_diag, unsigned long long* escapes, hipStream_t st);
hipError_t prepare_fused(int prec, int dim, size_t smem);
void launch_reduce_fields(const Tables& T, int prec, int dim, int nblocks, int with_rho,
                          double* out, hipStream_t st);
void launch_kinetic(const Tables& T, int prec, int dim, int nblocks, double* out,
                    hipStream_t st);
void launch_zero_doubles(double* p, int n, hipStream_t st);
void launch_diag_clear(const Tables& T, int nruns, hipStream_t st);
void launch_load_positions(const Tables& T, int prec, int dim, int nblocks, const double* x,
                           const double* y, const double* z, hipStream_t st);
void launch_store_positions(const Tables& T, int prec, int dim, int nblocks, double* x,
                            double* y, double* z, hipStream_t st);
size_t fused_smem_bytes(int prec, int dim, int tx, int ty, int tz, int halo, int with_rho);

}  // namespace lpic
