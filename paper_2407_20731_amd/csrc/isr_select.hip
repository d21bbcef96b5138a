// Order-independent kernels for gfx950: zero fill, threshold selection
// (level 1 on exponent bins, levels 2..6 on fraction bits, sort-resolve),
// and the finalize step.  The threshold rule (arXiv 2407.20731, Sec. IV-B
// reading): tau is the largest energy value v whose dropped energy
// S(v) = RN(exact sum of energies < v) does not exceed B = (tol*tol)*U2.
#include "isr.h"
#include "isr_fastsel.cuh"

namespace isr {

__global__ void k_zero(u64* p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0ull;
}

// Per-component state to mapped pinned host memory, written by the GPU (no
// DMA copy: a small copy would queue behind bulk transfers on the copy
// engines, e.g. a blob going to the lossless stage).
__global__ __launch_bounds__(64) void k_state_out(const u64* src, u64* dst, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += 64) dst[i] = src[i];
}

hipError_t launch_state_out(const CompState* src, CompState* host_dst, int ncomp, hipStream_t s) {
  void* d = nullptr;
  hipError_t e = hipHostGetDevicePointer(&d, host_dst, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_state_out, dim3(1), dim3(64), 0, s, (const u64*)src, (u64*)d,
                     (int)(sizeof(CompState) * ncomp / 8));
  return hipGetLastError();
}

__global__ __launch_bounds__(64) void k_err_total(Job j, double* err2_out) {
  const double e = wb_round(hist_total(j.histR + (size_t)blockIdx.x * HBINS));
  if (threadIdx.x == 0) err2_out[blockIdx.x] = e;
}

hipError_t launch_err_total(const Job& j, double* err2_out, hipStream_t s) {
  hipLaunchKernelGGL(k_err_total, dim3(j.ncomp), dim3(64), 0, s, j, err2_out);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  size_t nw = bytes / 8;
  if (nw == 0) return hipSuccess;
  int grid = (int)((nw + 255) / 256);
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, (u64*)p, nw);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_refine(Job j, int L) {
  __shared__ u64 h[RBINS][2];
  refine_body(j, blockIdx.y, L, h, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(64) void k_select1(Job j, int sample) { select1_body(j, blockIdx.x, sample); }

__global__ __launch_bounds__(256) void k_select(Job j, int L) {
  __shared__ SelLds S;
  select_body(j, blockIdx.x, L, S);
}

__global__ __launch_bounds__(64) void k_finalize(Job j) { finalize_body(j, blockIdx.x); }

// Per-phase launches of the streaming path's order-independent bodies
// (isr_fastsel.cuh).
__global__ __launch_bounds__(256) void k_gather(Job j) {
  __shared__ GatherLds X;
  gather_body(j, blockIdx.y, blockIdx.x, gridDim.x, X, false);
}

__global__ __launch_bounds__(256) void k_count(Job j) { count_body(j, blockIdx.y, blockIdx.x, gridDim.x); }

__global__ __launch_bounds__(256) void k_scan1(Job j) {
  __shared__ ScanLds X;
  scan1_body(j, blockIdx.y, blockIdx.x, gridDim.x, X);
}

// Per-component tails of the phases above and of the sample pass and pass B
// (one workgroup per component, after the phase's kernel).
__global__ __launch_bounds__(256) void k_gather_tail(Job j) { gather_tail(j, blockIdx.x); }

__global__ __launch_bounds__(64) void k_sample_tail(Job j) { select_sample_body(j, blockIdx.x); }

__global__ __launch_bounds__(256) void k_passB_tail(Job j) {
  __shared__ __int128 r3[4][3];
  passB_tail(j, blockIdx.x, r3);
  if (j.hs_out) {  // the component's final state straight to the mapped host copy
    __syncthreads();
    const u64* src = (const u64*)(j.st + blockIdx.x);
    u64* dst = (u64*)(j.hs_out + blockIdx.x);
    for (int i = threadIdx.x; i < (int)(sizeof(CompState) / 8); i += 256) dst[i] = src[i];
  }
}

__global__ __launch_bounds__(256) void k_scan2(Job j) {
  __shared__ ScanLds X;
  scan2_body(j, blockIdx.y, blockIdx.x, gridDim.x, X);
}

// The selection of level 3, then levels 4..NLEV in the same workgroup (one
// per component), each refinement followed by its selection.  From level 4 on,
// the lists hold the members of one level-3 sub-bin (a few entries, unless
// thousands of energies agree in their top 23 bits) and the selection has
// usually been resolved already, so one launch replaces seven.
__global__ __launch_bounds__(256) void k_select_rest(Job j) {
  __shared__ RefselLds X;
  const int comp = blockIdx.x;
  select_body(j, comp, 3, X.U.S);
  for (int L = 4; L <= NLEV; ++L) {
    __syncthreads();
    __threadfence();
    __syncthreads();
    if (j.st[comp].resolved) return;
    refine_body(j, comp, L, X.U.h, 0, 1);
    __syncthreads();
    __threadfence();
    __syncthreads();
    select_body(j, comp, L, X.U.S);
  }
}

// the refinement levels 2..NLEV: levels 2 and 3 (over list 0) as refinement
// kernels over the whole grid, the selections of level 2 and of the rest one
// workgroup per component
hipError_t launch_refsel(const Job& j, int gx, hipStream_t s) {
  hipLaunchKernelGGL(k_refine, dim3(gx, j.ncomp), dim3(256), 0, s, j, 2);
  hipLaunchKernelGGL(k_select, dim3(j.ncomp), dim3(256), 0, s, j, 2);
  // level 3 matches only the members of one level-2 sub-bin, so its
  // workgroups flush few bins: more of them, for fewer list loads each
  const int gx3 = gx * 8 < GATHER_GMAX ? gx * 8 : GATHER_GMAX;
  hipLaunchKernelGGL(k_refine, dim3(gx3, j.ncomp), dim3(256), 0, s, j, 3);
  hipLaunchKernelGGL(k_select_rest, dim3(j.ncomp), dim3(256), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_gather(const Job& j, int gx, hipStream_t s) {
  if (gx > GATHER_GMAX) gx = GATHER_GMAX;
  hipLaunchKernelGGL(k_gather, dim3(gx, j.ncomp), dim3(256), 0, s, j);
  hipLaunchKernelGGL(k_gather_tail, dim3(j.ncomp), dim3(256), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_count(const Job& j, int gx, hipStream_t s) {
  // independent atomics: many workgroups (four times the gather's; a few
  // list loads per lane each)
  hipLaunchKernelGGL(k_count, dim3(gx * 4, j.ncomp), dim3(256), 0, s, j);
  const int g = scan_grid_elems(j.n_elem);
  hipLaunchKernelGGL(k_scan1, dim3(g, j.ncomp), dim3(256), 0, s, j);
  hipLaunchKernelGGL(k_scan2, dim3(g, j.ncomp), dim3(256), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_select1(const Job& j, int sample, hipStream_t s) {
  hipLaunchKernelGGL(k_select1, dim3(j.ncomp), dim3(64), 0, s, j, sample);
  return hipGetLastError();
}

hipError_t launch_refine(const Job& j, int L, int gx, hipStream_t s) {
  hipLaunchKernelGGL(k_refine, dim3(gx, j.ncomp), dim3(256), 0, s, j, L);
  return hipGetLastError();
}

hipError_t launch_select(const Job& j, int L, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(j.ncomp), dim3(256), 0, s, j, L);
  return hipGetLastError();
}

hipError_t launch_finalize(const Job& j, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(j.ncomp), dim3(64), 0, s, j);
  return hipGetLastError();
}

}  // namespace isr

namespace isr {

int words_per_elem(int order) {
  const int n = order + 1, n3 = n * n * n;
  return (n3 + 63) / 64;
}

int tiles_per_comp(int order, long long n_elem) {
  const int n = order + 1, n2 = n * n;
  const int epi = 256 / n2 > 0 ? 256 / n2 : 1;
  return (int)((n_elem + epi - 1) / epi);
}

hipError_t launch_fast_tail(int kind, const Job& j, hipStream_t s) {
  if (kind == F_SAMPLE)
    hipLaunchKernelGGL(k_sample_tail, dim3(j.ncomp), dim3(64), 0, s, j);
  else if (kind == F_PASSB)
    hipLaunchKernelGGL(k_passB_tail, dim3(j.ncomp), dim3(256), 0, s, j);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fast(int kind, int precision, const Job& j, int gx, hipStream_t s) {
  if (j.tile > 0) {
    if (precision == ISR_PREC_FP32) return launch_dense_fp32(kind, j, gx, s);
    if (precision == ISR_PREC_BF16) return launch_dense_bf16(kind, j, gx, s);
    return hipErrorInvalidValue;
  }
  if (precision == ISR_PREC_FP64) return launch_fast_fp64(kind, j, gx, s);
  if (precision == ISR_PREC_FP32) return launch_fast_fp32(kind, j, gx, s);
  if (precision == ISR_PREC_BF16) return launch_fast_bf16(kind, j, gx, s);
  return hipErrorInvalidValue;
}

int resident_fast(int kind, int precision, int order, int tile) {
  static int cache[3][3][16];
  static int dcache[3][3][16][65];
  if (kind < 0 || kind > 2 || precision < 0 || precision > 2 || !fast_order(order, precision)) return 1;
  if (tile > 0) {
    if (precision == ISR_PREC_FP64 || tile > 64 || !dense_shape(order, tile)) return 1;
    int& d = dcache[kind][precision][order][tile];
    if (d == 0) d = precision == ISR_PREC_FP32 ? resident_dense_fp32(kind, order, tile) : resident_dense_bf16(kind, order, tile);
    return d;
  }
  int& c = cache[kind][precision][order];
  if (c == 0) {
    if (precision == ISR_PREC_FP64)
      c = resident_fast_fp64(kind, order);
    else if (precision == ISR_PREC_FP32)
      c = resident_fast_fp32(kind, order);
    else
      c = resident_fast_bf16(kind, order);
  }
  return c;
}

hipError_t launch_pass(int kind, int precision, const Job& j, int grid, hipStream_t s, void* extra, int extra_i) {
  if (precision == ISR_PREC_FP64) return launch_pass_fp64(kind, j, grid, s, extra, extra_i);
  if (precision == ISR_PREC_FP32) return launch_pass_fp32(kind, j, grid, s, extra, extra_i);
  if (precision == ISR_PREC_BF16) return launch_pass_bf16(kind, j, grid, s, extra, extra_i);
  return hipErrorInvalidValue;
}

int resident_blocks(int kind, int precision, int order) {
  static int cache[5][3][16];
  if (kind < 0 || kind > 4 || precision < 0 || precision > 2 || order < 1 || order > 15) return 1;
  int& c = cache[kind][precision][order];
  if (c == 0) {
    if (precision == ISR_PREC_FP64 || kind == K_DECOMP)
      c = resident_fp64(kind, order);
    else if (precision == ISR_PREC_FP32)
      c = resident_fp32(kind, order);
    else
      c = resident_bf16(kind, order);
  }
  return c;
}

}  // namespace isr

namespace isr {

hipError_t launch_fbatch(int precision, const BatchCtl& B, int grid, size_t lds_bytes, hipStream_t s) {
  if (precision == ISR_PREC_FP32) return launch_fbatch_fp32(B, grid, lds_bytes, s);
  if (precision == ISR_PREC_BF16) return launch_fbatch_bf16(B, grid, lds_bytes, s);
  return hipErrorInvalidValue;
}

size_t fbatch_lds(int precision, int order, int tile) {
  return precision == ISR_PREC_FP32 ? fbatch_lds_fp32(order, tile) : fbatch_lds_bf16(order, tile);
}

int fbatch_resident(int precision, size_t lds_bytes) {
  return precision == ISR_PREC_FP32 ? fbatch_resident_fp32(lds_bytes) : fbatch_resident_bf16(lds_bytes);
}

hipError_t launch_batch(int precision, const BatchCtl& B, int grid, size_t lds_bytes, hipStream_t s) {
  if (precision == ISR_PREC_FP64) return launch_batch_fp64(B, grid, lds_bytes, s);
  if (precision == ISR_PREC_FP32) return launch_batch_fp32(B, grid, lds_bytes, s);
  if (precision == ISR_PREC_BF16) return launch_batch_bf16(B, grid, lds_bytes, s);
  return hipErrorInvalidValue;
}

size_t batch_lds(int precision) {
  if (precision == ISR_PREC_FP64) return batch_lds_fp64();
  if (precision == ISR_PREC_FP32) return batch_lds_fp32();
  return batch_lds_bf16();
}

int batch_resident(int precision, size_t lds_bytes) {
  if (precision == ISR_PREC_FP64) return batch_resident_fp64(lds_bytes);
  if (precision == ISR_PREC_FP32) return batch_resident_fp32(lds_bytes);
  return batch_resident_bf16(lds_bytes);
}

}  // namespace isr
