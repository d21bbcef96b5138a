// Order-independent kernels for gfx950: zero fill, threshold selection
// (level 1 on exponent bins, levels 2..6 on fraction bits, sort-resolve),
// and the finalize step.  The threshold rule (arXiv 2407.20731, Sec. IV-B
// reading): tau is the largest energy value v whose dropped energy
// S(v) = RN(exact sum of energies < v) does not exceed B = (tol*tol)*U2.
#include "isr.h"
#include "isr_selbody.cuh"
#include "isr_xsum.cuh"

namespace isr {

__global__ void k_zero(u64* p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0ull;
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

// refine level L over the candidate lists, then (last workgroup of the
// component) the level-L selection
__global__ __launch_bounds__(256) void k_refsel(Job j, int L) {
  __shared__ union {
    u64 h[RBINS][2];
    SelLds S;
  } U;
  __shared__ int last;
  const int comp = blockIdx.y;
  if (j.st[comp].resolved) return;
  refine_body(j, comp, L, U.h, blockIdx.x, gridDim.x);
  if (!last_block(j.done + (D_REFSEL + L) * 8 + comp, &last, gridDim.x)) return;
  select_body(j, comp, L, U.S);
}

// ---- streaming path: exact window bins, exact totals, level-1 selection ------
// Every workgroup adds the significands of its share of list 0 (the window
// energies) to the window bins; workgroup 0 turns the per-workgroup integer
// sums of pass A into exact bins (norm terms anywhere, energies below the
// window in bins below it) and puts the count of energies above the window
// into bin win_hi; the last workgroup runs the level-1 selection.
__global__ __launch_bounds__(256) void k_gather(Job j) {
  __shared__ u64 red[4][9];
  __shared__ __int128 part[256];
  __shared__ int last;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int comp = blockIdx.y;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const int wlo = st->win_lo, whi = st->win_hi;
  HistBin* gE = j.histE + (size_t)comp * HBINS;
  HistBin* gN = j.histN + (size_t)comp * HBINS;
  const u64* list = list_ptr(j, comp, 0);
  const u64 nl = st->list_count[0] < j.list_cap ? st->list_count[0] : j.list_cap;
  u64 acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // (cnt, lo, hi) of the three window bins
  for (u64 i = (u64)blockIdx.x * 256 + tid; i < nl; i += (u64)gridDim.x * 256) {
    const u64 key = list[i];
    const int k = (int)(key >> 52) - wlo;  // 0..2; window bins are >= 1 (normal numbers)
    const u64 sig = (key & M52) | (1ull << 52);
    for (int b = 0; b < 3; ++b) {
      if (b == k) {
        acc[3 * b] += 1ull;
        acc[3 * b + 1] += sig & M21;
        acc[3 * b + 2] += sig >> 21;
      }
    }
  }
  for (int k = 0; k < 9; ++k) {
    const u64 w = wave_sum64(acc[k]);
    if (lane == 0) red[wv][k] = w;
  }
  __syncthreads();
  // per-workgroup partials (no contended atomics); the last workgroup adds them
  if (tid < 9) j.gslot[((size_t)comp * GATHER_GMAX + blockIdx.x) * 16 + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  if (blockIdx.x == 0) {
    // totals of pass A's workgroup sums: fields 0..2 norm, 3..5 energy, 6 count
    for (int f = 0; f < 7; ++f) {
      const __int128 t = block_total_rows(j.slotsA + (size_t)comp * j.gA * 8, j.gA, 8, f, part, tid);
      if (tid == 0) red[0][f] = (u64)t, red[1][f] = (u64)((unsigned __int128)t >> 64);
      __syncthreads();
    }
    if (tid == 0) {
      __int128 K[3];
      for (int k = 0; k < 3; ++k) K[k] = (__int128)(((unsigned __int128)red[1][k] << 64) | red[0][k]);
      emit_total(gN, K, st->xm_norm, j.xh, -1);
      for (int k = 0; k < 3; ++k) K[k] = (__int128)(((unsigned __int128)red[1][3 + k] << 64) | red[0][3 + k]);
      if (wlo < whi) emit_total(gE, K, wlo - 1023, j.xh, wlo - 1);
      const u64 above = red[0][6];
      if (above) atomicAdd(&gE[whi].cnt, above);
    }
  }
  if (!last_block(j.done + D_GATHER * 8 + comp, &last, gridDim.x)) return;
  for (int k = 0; k < 9; ++k) {
    const u64 w = (u64)block_total_rows((const long long*)j.gslot + (size_t)comp * GATHER_GMAX * 16, gridDim.x, 16,
                                        k, part, tid);
    const int b = wlo + k / 3;
    if (tid == 0 && w && b < whi) {
      if (k % 3 == 0) atomicAdd(&gE[b].cnt, w);
      if (k % 3 == 1) atomicAdd(&gE[b].lo, w);
      if (k % 3 == 2) atomicAdd(&gE[b].hi, w);
    }
  }
  __threadfence();
  __syncthreads();
  if (tid < 64) select1_body(j, comp, 0);
  __syncthreads();
  if (tid == 0) {
    // bound on the error terms of pass B: a little above the budget, or, when
    // everything is kept, a little above the rounding level of the transforms
    int m;
    if (st->B > 0.0) {
      m = ilogb(st->B) + 6;
    } else {
      const int eu = st->U2 > 0.0 ? ilogb(st->U2) : XM_MIN;
      m = eu - (j.precision == 0 ? 80 : 30);
    }
    st->xm_err = m < XM_MIN ? XM_MIN : (m > XM_MAX ? XM_MAX : m);
  }
}

// Per-element kept counts: pass A stored the count of energies above the
// window; every window entry of list 0 at or above tau adds one.
__global__ __launch_bounds__(256) void k_count(Job j) {
  const int tid = threadIdx.x;
  const int comp = blockIdx.y;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  u32* cnt = j.cnt + (size_t)comp * j.n_elem;
  const u64 tk = dbits(st->tau);
  const u64* list = list_ptr(j, comp, 0);
  const u32* lidx = j.lidx + (size_t)comp * j.list_cap;
  const u64 nl = st->list_count[0] < j.list_cap ? st->list_count[0] : j.list_cap;
  for (u64 i = (u64)blockIdx.x * 256 + tid; i < nl; i += (u64)gridDim.x * 256)
    if (list[i] >= tk) atomicAdd(&cnt[lidx[i]], 1u);
}

// Element offsets from the counts, in two steps over chunks of SCAN_CHUNK
// elements: chunk sums (the last workgroup turns them into chunk offsets and
// checks the total against the selected kept count), then a local scan of
// every chunk.
constexpr int SCAN_CHUNK = 1024;

DEV u64 block_excl_scan(u64 v, u64* part, int tid, u64* total) {
  part[tid] = v;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    const u64 o = tid >= d ? part[tid - d] : 0ull;
    __syncthreads();
    part[tid] += o;
    __syncthreads();
  }
  const u64 incl = part[tid];
  *total = part[255];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(256) void k_scan1(Job j) {
  __shared__ u64 part[256];
  __shared__ int last;
  const int tid = threadIdx.x;
  const int comp = blockIdx.y;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const long long E = j.n_elem;
  const u32* cnt = j.cnt + (size_t)comp * E;
  const long long nch = (E + SCAN_CHUNK - 1) / SCAN_CHUNK;
  u64* coff = j.chunk + (size_t)comp * j.nchunk;
  for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
    u64 v = 0;
    for (int k = 0; k < SCAN_CHUNK / 256; ++k) {
      const long long e = c * SCAN_CHUNK + k * 256 + tid;
      if (e < E) v += cnt[e];
    }
    u64 tot;
    (void)block_excl_scan(v, part, tid, &tot);
    if (tid == 0) coff[c] = tot;
  }
  if (!last_block(j.done + D_COUNT * 8 + comp, &last, gridDim.x)) return;
  // chunk sums -> exclusive chunk offsets (in place), total check
  u64 run = 0;
  for (long long c0 = 0; c0 < nch; c0 += 256) {
    const long long c = c0 + tid;
    const u64 v = c < nch ? coff[c] : 0ull;
    u64 tot;
    const u64 ex = block_excl_scan(v, part, tid, &tot);
    if (c < nch) coff[c] = run + ex;
    run += tot;
  }
  if (tid == 0) {
    j.elem_ptr[(size_t)comp * (E + 1) + E] = run;
    if (run != st->kept) atomicOr(&st->flags, ST_LIST);
  }
}

__global__ __launch_bounds__(256) void k_scan2(Job j) {
  __shared__ u64 part[256];
  const int tid = threadIdx.x;
  const int comp = blockIdx.y;
  CompState* st = j.st + comp;
  if (st->flags & ST_MISS) return;
  const long long E = j.n_elem;
  const u32* cnt = j.cnt + (size_t)comp * E;
  const long long nch = (E + SCAN_CHUNK - 1) / SCAN_CHUNK;
  const u64* coff = j.chunk + (size_t)comp * j.nchunk;
  u64* eptr = j.elem_ptr + (size_t)comp * (E + 1);
  for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
    // thread t owns elements c*CHUNK + 4t .. 4t+3
    const long long e0 = c * SCAN_CHUNK + 4 * tid;
    u32 v[4];
    u64 sum = 0;
    for (int k = 0; k < 4; ++k) {
      v[k] = e0 + k < E ? cnt[e0 + k] : 0u;
      sum += v[k];
    }
    u64 tot;
    u64 run = coff[c] + block_excl_scan(sum, part, tid, &tot);
    for (int k = 0; k < 4; ++k) {
      if (e0 + k < E) eptr[e0 + k] = run;
      run += v[k];
    }
  }
}

hipError_t launch_refsel(const Job& j, int L, int gx, hipStream_t s) {
  hipLaunchKernelGGL(k_refsel, dim3(gx, j.ncomp), dim3(256), 0, s, j, L);
  return hipGetLastError();
}

hipError_t launch_gather(const Job& j, int gx, hipStream_t s) {
  if (gx > GATHER_GMAX) gx = GATHER_GMAX;
  hipLaunchKernelGGL(k_gather, dim3(gx, j.ncomp), dim3(256), 0, s, j);
  return hipGetLastError();
}

hipError_t launch_count(const Job& j, int gx, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(gx, j.ncomp), dim3(256), 0, s, j);  // independent atomics: many workgroups
  const long long nch = (j.n_elem + SCAN_CHUNK - 1) / SCAN_CHUNK;
  const int g = (int)(nch < 1024 ? nch : 1024);
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
  if (kind == K_DECOMP || precision == ISR_PREC_FP64) return launch_pass_fp64(kind, j, grid, s, extra, extra_i);
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
