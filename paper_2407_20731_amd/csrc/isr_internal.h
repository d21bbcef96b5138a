// Internal definitions shared by the HIP kernels and the host runtime.
// Nothing here is part of the public ABI (include/isr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace isr {

typedef unsigned long long u64;
typedef unsigned int u32;

// ---- exact sums of non-negative FP64 terms ------------------------------
// A term v = sig * 2^(max(E,1) - 1075) (E = biased exponent field, sig = 53-bit
// significand with its implicit bit) is kept as an integer in units of 2^-1075
// ("X units"): X(v) = sig << max(E,1).  Terms are binned by E; a bin stores
// the count and the exact sum of its significands split as hi * 2^21 + lo,
// hi summing sig >> 21 (< 2^32) and lo summing sig & (2^21 - 1).  Bin 2047
// (Inf/NaN) only ever counts, and flags a non-finite input.
constexpr int HBINS = 2048;
struct HistBin {
  u64 cnt, lo, hi;
};

// LDS window of exponent bins held by one workgroup (values outside go
// straight to the global bins).
constexpr int WIN = 256;
constexpr int WIN_HEAD = 16;  // bins kept above the first tile's largest exponent

// Refinement of the threshold inside the boundary exponent bin: the 52
// fraction bits are resolved 11 at a time (bits 51..41, 40..30, 29..19,
// 18..8), then 8 (bits 7..0).  Levels are numbered 2..6; level 1 is the
// exponent.
constexpr int RBINS = 2048;
constexpr int NLEV = 6;
constexpr int CAP = 4096;  // a sub-bin with at most CAP members is resolved by sorting

__host__ __device__ constexpr int level_shift(int L) { return L == 6 ? 0 : 41 - 11 * (L - 2); }
__host__ __device__ constexpr int level_bits(int L) { return L == 6 ? 8 : 11; }

// Per-component selection state, written by the select kernels.
struct alignas(256) CompState {
  u64 P1[64];         // exact sum (X units) of all energies below the boundary bin
  double U2, B, tau, dropped, err2, rel;
  double tol;
  u64 n_values;       // values in this component
  u64 kept;           // final kept count
  u64 kept_above;     // energies above the current bin / sub-bin
  u64 key_prefix;     // bits fixed so far (of the FP64 pattern of tau)
  u64 key_mask;
  u64 cur_count;      // members of the current bin / sub-bin
  u64 r_lo, r_hi;     // 128-bit slack, in significand units of the boundary bin
  u64 w_lo, w_hi;     // 128-bit significand sum dropped inside the boundary bin
  u64 list_count[3];  // candidate list fill levels
  int32_t bstar;      // boundary exponent bin, -1 when tau is +inf or 0
  int32_t level;      // last level decided
  int32_t resolved;   // tau final
  int32_t flags;      // ST_* below
  int32_t win_lo;     // exponent bins [win_lo, win_hi) captured speculatively
  int32_t win_hi;     //   by pass 1 (empty when win_lo >= win_hi)
  int32_t need_pass2; // boundary bin outside the window: run the candidate pass
  int32_t list0_exact;  // list 0 holds exactly the boundary bin's energies
  // streaming path (isr_engine.cuh): the energy histogram holds exact sums
  // only inside the window, everything below it as one exact total
  int32_t win_mode;
  int32_t xm_norm;    // log2 of the bound on norm terms used by the extraction sums
  int32_t xm_err;     // same for the error terms
  int32_t samp_maxe;  // largest biased exponent of a sampled norm term
  double samp_u2;     // sampled norm terms (rounded sum, only to place the window)
};

enum : int32_t {
  ST_NONFINITE = 1,   // Inf/NaN in the field
  ST_OVERFLOW = 2,    // an energy or norm term overflowed FP64
  ST_SPIN = 4,        // a bounded wait expired (should never happen)
  ST_LIST = 8,        // a candidate list overflowed its capacity
  ST_MISS = 16,       // streaming path: tau outside the sampled window (the
                      // general pipeline runs instead; not an error)
};

struct DevTables {
  const double* A;    // [n][n]  A[p][i]
  const double* V;    // [n][n]  V[i][k]
  const double* w3;   // [n][n][n]
  const double* g3;   // [n][n][n]
  const float* A32;   // FP32 roundings (mixed paths)
  const float* V32;
};

// Everything one compression needs on the device.
struct Job {
  const double* u;     // field
  const double* jac;   // per-element Jacobian or null
  long long comp_stride;
  long long n_elem;
  int order;
  int ncomp;
  int precision;
  int vbytes;          // 8 (FP64 values) or 4
  double tol;
  double cut_scale;    // the cut's budget is ((tol*tol)*U2)*cut_scale (1: the whole budget)
  double Bov[8];       // per-component budget override (repair); < 0 = none
  DevTables tab;
  // scratch
  HistBin* histE;      // [ncomp][HBINS]  energies
  HistBin* histN;      // [ncomp][HBINS]  norm terms
  HistBin* histR;      // [ncomp][HBINS]  error terms
  HistBin* histL;      // [NLEV-1][ncomp][RBINS]  refinement levels 2..6
  HistBin* histEs;     // [ncomp][HBINS]  energies of the sampled tiles
  HistBin* histNs;     // [ncomp][HBINS]  norm terms of the sampled tiles
  long long sample_stride;  // every sample_stride-th tile is sampled; 0 = no sample pass
  CompState* st;       // [ncomp]
  CompState* hs_out;   // streaming path: device address of the request's mapped host copy of st, written by
                       // pass B's tail; null = a separate copy kernel after the pipeline
  u64* lists;          // [ncomp][3][list_cap]
  u64 list_cap;
  // streaming path
  u32* lidx;           // [ncomp][list_cap] element of each list-0 entry
  u32* cnt;            // [ncomp][n_elem] kept coefficients per element
  long long* slotsA;   // [ncomp][gA][8] per-workgroup exact partial sums
  long long* slotsB;   // [ncomp][gB][4]
  u32* done;           // [16][8] finished-workgroup counters
  u64* chunk;          // [ncomp][nchunk] element-offset scan: chunk sums, then offsets
  long long nchunk;
  int gA, gB;          // workgroups per component of the two streaming passes
  int xh;              // extraction headroom (log2 of twice the terms per lane)
  int tile;            // elements per wavefront tile of the dense-tile engine; 0 = wave-tile engine
  u64* lookback;       // [ncomp][tiles]
  u32* ticket;         // [4]
  // blob (device)
  u64* bitmap;         // [ncomp][n_elem][W]
  u64* elem_ptr;       // [ncomp][n_elem + 1]
  void* values;        // kept values, component after component
  u64* voff;           // [ncomp] offset of each component's first value
  // quantised variant: per-component step of the codes (device), and the
  // codes written by the quantisation pass (FP32 integers, values' layout)
  const double* qstep;
  float* qvals;
  // per-element cut: the threshold of every element ([ncomp][n_elem]); null
  // = the component's threshold st[comp].tau
  const double* tau_elem;
};

// Persistent batch launch (isr_batch.cuh): phases of the shared work queue.
enum BatchPhase {
  PH_P0 = 0, PH_S0, PH_P1, PH_S1, PH_P2,
  PH_R2, PH_S2, PH_R3, PH_S3, PH_R4, PH_S4, PH_R5, PH_S5, PH_R6, PH_S6,
  PH_P3, PH_FIN, NPH
};
struct BatchCtl {
  const Job* jobs;          // [nsnap], device
  const int* pair_snap;     // [npairs] snapshot of each (snapshot, component) pair
  const int* pair_comp;     // [npairs]
  const long long* items;   // [NPH][npairs + 1]: prefix of item counts over pairs
  long long phase_off[NPH + 1];  // first ticket of each phase
  int npairs;
  u32* done;                // [NPH][npairs] completed items
  unsigned long long* ticket;
  int* err;                 // a bounded wait expired
};
hipError_t launch_batch(int precision, const BatchCtl& B, int grid, size_t lds_bytes, hipStream_t s);
size_t batch_lds(int precision);
int batch_resident(int precision, size_t lds_bytes);
hipError_t launch_batch_fp64(const BatchCtl& B, int grid, size_t lds, hipStream_t s);
hipError_t launch_batch_fp32(const BatchCtl& B, int grid, size_t lds, hipStream_t s);
hipError_t launch_batch_bf16(const BatchCtl& B, int grid, size_t lds, hipStream_t s);
size_t batch_lds_fp64();
size_t batch_lds_fp32();
size_t batch_lds_bf16();
int batch_resident_fp64(size_t lds);
int batch_resident_fp32(size_t lds);
int batch_resident_bf16(size_t lds);

// Streaming passes (isr_passes.cuh), one instantiation file per precision.
enum PassKind { K_PASS1 = 0, K_PASS2 = 1, K_PASS3 = 2, K_DECOMP = 3, K_FORWARD = 4, K_QUANT = 5 };
int tiles_per_comp(int order, long long n_elem);
int words_per_elem(int order);
// grid: x extent (pass1/pass2 also get y = ncomp); extra: output pointer of
// K_FORWARD / K_DECOMP; extra_i: K_DECOMP writes FP64 (1) or FP32 (0)
hipError_t launch_pass(int kind, int precision, const Job& j, int grid, hipStream_t s, void* extra = nullptr,
                       int extra_i = 0);
int resident_blocks(int kind, int precision, int order);  // workgroups per CU
hipError_t launch_pass_fp64(int kind, const Job& j, int grid, hipStream_t s, void* extra, int extra_i);
hipError_t launch_pass_fp32(int kind, const Job& j, int grid, hipStream_t s, void* extra, int extra_i);
hipError_t launch_pass_bf16(int kind, const Job& j, int grid, hipStream_t s, void* extra, int extra_i);
int resident_fp64(int kind, int order);
int resident_fp32(int kind, int order);
int resident_bf16(int kind, int order);
// order-independent kernels (isr_select.hip)
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// copy of the per-component states into mapped pinned host memory (host_dst
// from hipHostMalloc with hipHostMallocMapped), by a kernel
hipError_t launch_state_out(const CompState* src, CompState* host_dst, int ncomp, hipStream_t s);
// correctly rounded exact totals of the error histograms j.histR, per
// component, into err2_out[ncomp] (device)
hipError_t launch_err_total(const Job& j, double* err2_out, hipStream_t s);
// per-element cut (isr_elemcut.hip): every element's threshold into
// tau[ncomp][n_elem] from the FP64 coefficients coef (isr_forward's layout),
// at budgets ((tol*tol)*U2_e)*scale[comp]; the component totals (U2, the
// dropped energy) and kept counts into j.st.  G: zeroed digit totals of
// elemcut_digit_bytes(ncomp) bytes; j.st[*].kept and flags start at 0.
hipError_t launch_elemcut(const Job& j, const double* coef, double* tau, u64* G, const double* scale, int grid,
                          hipStream_t s);
size_t elemcut_digit_bytes(int ncomp);
hipError_t launch_select1(const Job& j, int sample, hipStream_t s);
hipError_t launch_refine(const Job& j, int level, int grid_x, hipStream_t s);
hipError_t launch_select(const Job& j, int level, hipStream_t s);
hipError_t launch_finalize(const Job& j, hipStream_t s);
hipError_t launch_refsel(const Job& j, int grid_x, hipStream_t s);  // levels 2..NLEV

// Streaming path (isr_engine.cuh) for orders 1..7.
enum FastKind { F_SAMPLE = 0, F_PASSA = 1, F_PASSB = 2 };
enum DoneSlot { D_SAMPLE = 0, D_GATHER = 1, D_COUNT = 2, D_PASSB = 3, D_REFSEL = 4 };  // D_REFSEL + level
constexpr int FAST_MAX_ORDER = 7;     // every precision
constexpr int FAST_MAX_ORDER_MF = 11; // FP32 / BF16 (large-order engine, isr_engine_l.cuh)
inline bool fast_order(int order, int precision) {
  return order >= 1 && (order <= FAST_MAX_ORDER || (precision != 0 && order <= FAST_MAX_ORDER_MF));
}
// Tile shapes compiled for the dense-tile engine (isr_engine_d.cuh, FP32 and
// BF16): X(order, elements per wavefront tile).
#define ISR_DENSE_SHAPES(X)                                                                               \
  X(1, 32) X(1, 64) X(2, 16) X(2, 32) X(3, 4) X(3, 8) X(4, 4) X(4, 8) X(5, 2) X(5, 4) X(5, 8) X(6, 1) X(6, 2) \
  X(6, 3) X(7, 1) X(7, 2) X(8, 1) X(8, 2) X(9, 1) X(9, 2) X(10, 1) X(11, 1)
inline bool dense_shape(int order, int tile) {
#define ISR_SHAPE_IS(O, T) \
  if (order == O && tile == T) return true;
  ISR_DENSE_SHAPES(ISR_SHAPE_IS)
#undef ISR_SHAPE_IS
  return false;
}
// candidate tiles of one order for the autotuner: 0 (the wave-tile engine,
// orders 1..11) first, then the compiled dense shapes; returns the count
inline int tile_candidates(int order, int* out, int cap) {
  int k = 0;
  if (order >= 1 && order <= FAST_MAX_ORDER_MF && k < cap) out[k++] = 0;
#define ISR_SHAPE_ADD(O, T) \
  if (order == O && k < cap) out[k++] = T;
  ISR_DENSE_SHAPES(ISR_SHAPE_ADD)
#undef ISR_SHAPE_ADD
  return k;
}
// built-in choice before any tuning (measured on MI355X, BF16, tol 1e-3)
inline int default_tile(int order, int precision) {
  if (precision == 0 || order < 1 || order > FAST_MAX_ORDER_MF) return 0;
  static const int t[12] = {0, 32, 16, 8, 4, 4, 2, 0, 1, 1, 1, 1};
  return t[order];
}
// elements per tile of the streaming path: the dense tile, else 64 / (N+1)^2
// (one from N = 7 up)
inline long long fast_epw(int order, int tile) {
  if (tile > 0) return tile;
  const long long n = order + 1;
  return 64 / (n * n) > 0 ? 64 / (n * n) : 1;
}
// values per lane per tile (norm terms of pass A, error terms of pass B)
inline long long fast_lane_terms(int order, int tile) {
  const long long n = order + 1;
  if (tile > 0) return (tile * n * n * n + 63) / 64;
  return n <= 8 ? 8 : (n * n * n + 63) / 64;
}
constexpr int FAST_GMAX = 2048;  // workgroups per component of a streaming pass
constexpr int GATHER_GMAX = 256;  // workgroups per component of the window-bin gather
hipError_t launch_fast(int kind, int precision, const Job& j, int grid_x, hipStream_t s);
// per-component tail of the sample pass (window selection) or of pass B
// (error total and final statistics), after that pass
hipError_t launch_fast_tail(int kind, const Job& j, hipStream_t s);
int resident_fast(int kind, int precision, int order, int tile);
hipError_t launch_dense_fp32(int kind, const Job& j, int grid_x, hipStream_t s);
hipError_t launch_dense_bf16(int kind, const Job& j, int grid_x, hipStream_t s);
int resident_dense_fp32(int kind, int order, int tile);
int resident_dense_bf16(int kind, int order, int tile);
hipError_t launch_fast_fp64(int kind, const Job& j, int grid_x, hipStream_t s);
hipError_t launch_fast_fp32(int kind, const Job& j, int grid_x, hipStream_t s);
hipError_t launch_fast_bf16(int kind, const Job& j, int grid_x, hipStream_t s);
int resident_fast_fp64(int kind, int order);
int resident_fast_fp32(int kind, int order);
int resident_fast_bf16(int kind, int order);
// Decompression of FP32 / BF16 blobs with the inverse of the engine that made
// them (the reconstruction pass B measured): wave-tile or large-order engine
// (tile 0, by order), or dense-tile engine (j.tile).
enum BlobEngine { ENG_GENERAL = 0, ENG_WAVE = 1, ENG_DENSE = 2 };
hipError_t launch_decomp_wave_fp32(const Job& j, int gx, hipStream_t s, void* out, int out_fp64);
hipError_t launch_decomp_wave_bf16(const Job& j, int gx, hipStream_t s, void* out, int out_fp64);
hipError_t launch_decomp_dense_fp32(const Job& j, int gx, hipStream_t s, void* out, int out_fp64);
hipError_t launch_decomp_dense_bf16(const Job& j, int gx, hipStream_t s, void* out, int out_fp64);
hipError_t launch_gather(const Job& j, int grid_x, hipStream_t s);
hipError_t launch_count(const Job& j, int grid_x, hipStream_t s);
constexpr int SCAN_CHUNK = 1024;  // elements per chunk of the element-offset scan
inline int scan_grid_elems(long long n_elem) {  // its workgroups per component
  const long long nch = (n_elem + SCAN_CHUNK - 1) / SCAN_CHUNK;
  return (int)(nch < 1024 ? nch : 1024);
}

// Persistent batch launch of the streaming path (isr_fbatch.cuh, FP32 and
// BF16): its phases, in queue order, and the (order, tile) shapes it holds:
// every candidate of the autotuner for orders 5, 7 and 9.
enum FastBatchPhase {
  FQ_SAMPLE = 0, FQ_PASSA, FQ_GATHER, FQ_R2, FQ_R3, FQ_R4, FQ_R5, FQ_R6, FQ_COUNT, FQ_SCAN1, FQ_SCAN2, FQ_PASSB, NFQ
};
static_assert(NFQ <= NPH, "phase offsets of BatchCtl");
#define ISR_FBATCH_SHAPES(X) X(5, 0) X(5, 2) X(5, 4) X(5, 8) X(7, 0) X(7, 1) X(7, 2) X(9, 0) X(9, 1) X(9, 2)
inline bool fbatch_shape(int order, int tile) {
#define ISR_FB_IS(O, T) \
  if (order == O && tile == T) return true;
  ISR_FBATCH_SHAPES(ISR_FB_IS)
#undef ISR_FB_IS
  return false;
}
constexpr int FBATCH_MIN = 8;  // smallest FP32 / BF16 batch that takes the persistent launch
hipError_t launch_fbatch(int precision, const BatchCtl& B, int grid, size_t lds_bytes, hipStream_t s);
size_t fbatch_lds(int precision, int order, int tile);
int fbatch_resident(int precision, size_t lds_bytes);
hipError_t launch_fbatch_fp32(const BatchCtl& B, int grid, size_t lds, hipStream_t s);
hipError_t launch_fbatch_bf16(const BatchCtl& B, int grid, size_t lds, hipStream_t s);
size_t fbatch_lds_fp32(int order, int tile);
size_t fbatch_lds_bf16(int order, int tile);
int fbatch_resident_fp32(size_t lds);
int fbatch_resident_bf16(size_t lds);

// Allocation-free entry point (isr_noalloc.hip): header bytes of a
// serialized blob (64 + 72 per component) written by a kernel, and the
// per-device lookup of the fixed scratch array's address.
constexpr int ISR_NOALLOC_HDR_MAX = 64 + 72 * 8;
hipError_t launch_put_bytes(const void* src, int n, void* dst, hipStream_t s);
int noalloc_init(int device);

// Host tables (isr_tables.cpp): correctly rounded FP64 values.
struct HostTables {
  int N;
  double xi[16], w[16], gamma[16];
  double V[256], A[256];
  double w3[4096], g3[4096];
};
bool host_tables(int N, HostTables* t);

}  // namespace isr
