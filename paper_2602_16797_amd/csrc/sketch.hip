// Sketch Y = S*A for the SparseStack embedding S (paper Sec. 2.2).
//
// S = zeta^{-1/2} [s_1 ... s_m]; column s_i has one +-1 in each of zeta pieces.
// Counter spec (shared in writing with the host oracle, not in code):
//   len_j = floor(d/zeta) + (j < d mod zeta), start_j = sum_{l<j} len_l
//   h(i,j) = splitmix64(seed ^ splitmix64(i*zeta + j))        (uint64 wrap)
//   row = start_j + ((h & 0xffffffff) * len_j >> 32),  sign = bit63 ? -1 : +1
// The +-1 rows are added exactly and the factor zeta^{-1/2} is applied once.
//
// Data layout: A is row-major with leading dimension lda (in elements); a
// complex A is read as 2n real columns (the sketch is real-linear), so both
// scalar types share one kernel over doubles.
//
// Kernel 1 (partial): grid (column tiles, row chunks).  A block owns a tile of
// CT double-columns and a chunk of rows and keeps the whole d x CT slice of Y
// in LDS (row stride CT + 1, so the 64/CT row slots of one instruction fall
// on different banks).  Wave w owns pieces w, w+8, ..., whose rows of Y no
// other wave touches; within a wave the row slots of one instruction may hit
// the same word, so the adds are LDS atomics (issued without waiting, unlike a
// read-modify-write).  Each lane hashes one row of the next 64 for the wave's
// piece while those rows load, and the targets are read with a cross-lane
// shuffle, so every (row, piece) pair is hashed once per tile.
// Kernel 2 (reduce): sums the chunk partials in chunk order and writes Y
// column-major (the layout of the QR that follows), flagging NaN/Inf.
// Both kernels take the accumulator type: FP64, or FP32 for the
// reduced-precision sketch (A is read in FP64 and rounded once per entry).
#include "common.hpp"
#include "kernels.hpp"

namespace rl {

__device__ inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// a with its sign flipped when the top bit of pk is set
__device__ inline double flip_sign(double a, int pk) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(a) ^ ((unsigned long long)((unsigned)pk & 0x80000000u) << 32);
  return __longlong_as_double((long long)b);
}
__device__ inline float flip_sign(float a, int pk) {
  return __int_as_float(__float_as_int(a) ^ (int)((unsigned)pk & 0x80000000u));
}

template <int CT, typename Acc>
__global__ __launch_bounds__(512) void k_sketch_partial(
    const double* __restrict__ A, int64_t lda_d, int64_t m, int64_t ncols_d, int d, int zeta,
    uint64_t seed, int64_t rows_per_chunk, Acc* __restrict__ part) {
  extern __shared__ double acc_raw[];
  // d x CT accumulators with a row stride of CT + 1, so the target rows of
  // the RS row slots of one instruction fall on different LDS banks
  constexpr int CTP = CT + 1;
  Acc* acc = reinterpret_cast<Acc*>(acc_raw);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = wave_index(), nwaves = blockDim.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * CT;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < m) ? r0 + rows_per_chunk : m;
  for (int i = tid; i < d * CTP; i += blockDim.x) acc[i] = (Acc)0;
  __syncthreads();
  constexpr int RS = 64 / CT;   // rows per instruction
  constexpr int NQ = 64 / RS;   // instructions per 64 rows
  const int slot = lane / CT, col = lane % CT;
  const bool colok = (c0 + col) < ncols_d;
  const int base = d / zeta, extra = d % zeta;
  for (int p = wave; p < zeta; p += nwaves) {
    const int len = base + (p < extra ? 1 : 0);
    const int start = p * base + (p < extra ? p : extra);
    // lane l hashes row g + l for piece p; the target's LDS offset (row times
    // CT + 1) and the sign travel as one word (sign in the top bit)
    auto target = [&](int64_t g) {
      const uint64_t i = (uint64_t)(g + lane);
      const uint64_t h = splitmix64(seed ^ splitmix64(i * (uint64_t)zeta + (uint64_t)p));
      const int tgt = start + (int)(((h & 0xFFFFFFFFull) * (uint64_t)len) >> 32);
      const int off = tgt * CTP;
      return (h >> 63) ? (off | (int)0x80000000) : off;
    };
    auto load = [&](Acc (&a)[NQ], int64_t g) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int64_t row = g + q * RS + slot;
        a[q] = (Acc)((row < r1 && colok) ? A[row * lda_d + c0 + col] : 0.0);
      }
    };
    // the next 64 rows are loaded and hashed while the current ones are added
    Acc an[NQ];
    load(an, r0);
    int pn = target(r0);
    for (int64_t g0 = r0; g0 < r1; g0 += 64) {
      Acc a[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) a[q] = an[q];
      const int packed = pn;
      if (g0 + 64 < r1) {
        load(an, g0 + 64);
        pn = target(g0 + 64);
      }
      // all targets first, then the adds back to back: a shuffle placed
      // between two adds would wait for the earlier add to finish.  Rows
      // past the chunk and columns past the tile hold zeros (see load), so
      // their adds change nothing and need no guard.
      int pk[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) pk[q] = __shfl(packed, q * RS + slot, WAVE);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const unsigned off = (unsigned)(pk[q] & 0x7FFFFFFF) + (unsigned)col;
        atomicAdd(&acc[off], flip_sign(a[q], pk[q]));
      }
    }
  }
  __syncthreads();
  Acc* out = part + (int64_t)blockIdx.y * d * ncols_d;
  for (int i = tid; i < d * CT; i += blockDim.x) {
    const int r = i / CT, c = i % CT;
    if (c0 + c < ncols_d) out[(int64_t)r * ncols_d + c0 + c] = acc[r * CTP + c];
  }
}

// Y (column-major, ld = d, element size es scalars) = scale * sum over chunks.
template <typename Acc>
__global__ void k_sketch_reduce(const Acc* __restrict__ part, int nchunk, int d, int64_t ncols_d, int es,
                                double scale, Acc* __restrict__ Ycol, Ctl* ctl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)d * ncols_d;
  if (idx >= total) return;
  const int64_t r = idx / ncols_d, cdb = idx % ncols_d;
  Acc s = (Acc)0;
  for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * total + idx];
  s *= (Acc)scale;
  if (!isfinite((double)s) && ctl) atomicOr(&ctl->nonfinite, 1);
  const int64_t elem = cdb / es, comp = cdb % es;
  Ycol[(elem * d + r) * es + comp] = s;
}

// widest column tile (in scalars) whose d x (CT + 1) slice of accumulators
// fits the LDS budget.  At d = 800 (n = 200) a 16-column tile (109 KB, one
// workgroup per CU) takes 1.39 ms against 1.64 ms for two workgroups of 8
// columns: each (row, piece) target is hashed once per 16 columns instead of
// once per 8, and one add instruction spans 4 rows of Y instead of 8, so
// fewer of its lanes meet on one LDS bank.
int sketch_plan_ct(int d, int64_t lds_budget, int acc_bytes) {
  const int cts[5] = {16, 8, 4, 2, 1};
  for (int c : cts)
    if ((int64_t)d * (c + 1) * acc_bytes <= lds_budget) return c;
  return 0;
}

// Accumulator elements of the chunk partials (the buffer holds doubles; FP32
// accumulators use the first half).
int64_t sketch_partial_doubles(int64_t m, int64_t ncols_d, int d, int64_t lds_budget, int* nchunk_out,
                               int64_t* rows_out, int acc_bytes) {
  const int ct = sketch_plan_ct(d, lds_budget, acc_bytes);
  if (ct == 0) return -1;
  const int64_t ntiles = (ncols_d + ct - 1) / ct;
  int64_t nchunk = (1024 + ntiles - 1) / ntiles;
  if (nchunk < 1) nchunk = 1;
  int64_t rows = (m + nchunk - 1) / nchunk;
  rows = ((rows + 63) / 64) * 64;
  if (rows < 64) rows = 64;
  nchunk = (m + rows - 1) / rows;
  if (nchunk < 1) nchunk = 1;
  *nchunk_out = (int)nchunk;
  *rows_out = rows;
  return nchunk * (int64_t)d * ncols_d;
}

template <int CT, typename Acc>
static hipError_t launch_partial(hipStream_t st, dim3 grid, size_t lds, const double* A, int64_t lda_d,
                                 int64_t m, int64_t ncols_d, int d, int zeta, uint64_t seed, int64_t rows,
                                 Acc* part) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)k_sketch_partial<CT, Acc>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_sketch_partial<CT, Acc>), grid, dim3(512), lds, st, A, lda_d, m, ncols_d, d, zeta, seed,
                     rows, part);
  return hipGetLastError();
}

template <typename Acc>
static hipError_t sketch_impl(hipStream_t st, const double* A, int64_t lda_d, int64_t m, int64_t ncols_d, int es,
                              int d, int zeta, uint64_t seed, double scale, Acc* part, Acc* Ycol, Ctl* ctl,
                              int64_t lds_budget) {
  int nchunk;
  int64_t rows;
  const int ab = (int)sizeof(Acc);
  if (sketch_partial_doubles(m, ncols_d, d, lds_budget, &nchunk, &rows, ab) < 0) return hipErrorInvalidValue;
  const int ct = sketch_plan_ct(d, lds_budget, ab);
  const int64_t ntiles = (ncols_d + ct - 1) / ct;
  dim3 grid((unsigned)ntiles, (unsigned)nchunk);
  const size_t lds = (size_t)d * (ct + 1) * sizeof(Acc);
  hipError_t e;
  switch (ct) {
    case 16: e = launch_partial<16, Acc>(st, grid, lds, A, lda_d, m, ncols_d, d, zeta, seed, rows, part); break;
    case 8: e = launch_partial<8, Acc>(st, grid, lds, A, lda_d, m, ncols_d, d, zeta, seed, rows, part); break;
    case 4: e = launch_partial<4, Acc>(st, grid, lds, A, lda_d, m, ncols_d, d, zeta, seed, rows, part); break;
    case 2: e = launch_partial<2, Acc>(st, grid, lds, A, lda_d, m, ncols_d, d, zeta, seed, rows, part); break;
    default: e = launch_partial<1, Acc>(st, grid, lds, A, lda_d, m, ncols_d, d, zeta, seed, rows, part); break;
  }
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)d * ncols_d;
  hipLaunchKernelGGL(k_sketch_reduce<Acc>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, part, nchunk,
                     d, ncols_d, es, scale, Ycol, ctl);
  return hipGetLastError();
}

hipError_t launch_sketch(hipStream_t st, const double* A, int64_t lda_d, int64_t m, int64_t ncols_d, int es, int d,
                         int zeta, uint64_t seed, double scale, void* part, void* Ycol, Ctl* ctl,
                         int64_t lds_budget, bool fp32) {
  if (fp32)
    return sketch_impl<float>(st, A, lda_d, m, ncols_d, es, d, zeta, seed, scale, (float*)part, (float*)Ycol, ctl,
                              lds_budget);
  return sketch_impl<double>(st, A, lda_d, m, ncols_d, es, d, zeta, seed, scale, (double*)part, (double*)Ycol, ctl,
                             lds_budget);
}

}  // namespace rl
