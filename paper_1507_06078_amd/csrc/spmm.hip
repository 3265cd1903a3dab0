// Fused filter SpMM for gfx950: one degree of the polynomial accelerator
// (the loop body of Algorithm 7, a factor of the product form of psi_d, and
// the plain products A*X of the Krylov augmentation [X, AX, ..., A^p X] of
// eq. S:ARR):
//
//   Yout = alpha * A * Yin + beta * Yin + gamma * Z      (Z optional)
//
// Design (about 1.5 flop per byte; bound by the memory system):
//  * matrix format (built on the host at set-up): one record of 8 values per
//    row {A[i][i-1], A[i][i], A[i][i+1], f0, f1, f2, f3, 0} with the columns
//    of the first four other ("far") entries in a table of 4 per row (unused
//    slots: column i, value 0); far entries past the fourth go to an overflow
//    CSR. A row's coefficients are one 64-byte scalar load;
//  * a wave visits a run of kRun consecutive rows and keeps Yin rows i-1, i,
//    i+1 in a register window, so the band and the beta*Yin term cost one new
//    Yin row per output row;
//  * inside a run the loads are software pipelined: columns two rows ahead,
//    the far gathers and the next window row one row ahead, so about twenty
//    loads per wave are in flight while a row is combined. Full runs take a
//    straight-line path with unconditional loads (the wait counts stay
//    exact); the first and last runs take a guarded row-at-a-time path;
//  * rows are read and written through buffer resources sized to the block
//    width: lanes past it read zeros and their stores are dropped, so no lane
//    predicate splits the code; lane l owns columns l, l+64, ... (FP32 blocks
//    with 16-byte aligned rows: 4 consecutive columns per lane, one 16-byte
//    load; FP64 blocks in the paired form: 2 consecutive columns per lane),
//    so every gathered row is read as full contiguous segments;
//  * the recurrence (beta*Yin + gamma*Z) is applied in the epilogue, so a
//    degree makes exactly one pass over Yin (gathered), Z and Yout;
//  * optional epilogue: per-workgroup column sums of squares of Yout in FP64,
//    reduced later in a fixed order (deterministic column norms for the
//    multi-power normalization);
//  * XCD-aware order: workgroup b runs on XCD b % 8; runs are dealt to the
//    XCDs in chunks of up to kMaxChunk consecutive runs, so that all XCDs
//    sweep the matrix together while a run's neighbours one grid line away
//    were mostly loaded by the same XCD (hits in its own L2). The chunk is the
//    largest power of two up to kMaxChunk dividing the waves per XCD, so the
//    first sweep of the waves covers whole chunks;
//  * paired form, for matrices with a frequent far offset P (grid operators:
//    the neighbour one grid line away): a wave processes rows i and i + P
//    together, and each row's entry in the other row's column is served from
//    the other run's register window. The kernel is limited by the rows
//    moved through each CU's vector memory path (six per output row in the
//    plain form for a 3D 7-point operator: one window row, four gathers, one
//    store), and the pairing drops one of the six.
#include <algorithm>
#include <climits>
#include <exception>
#include <map>

#include "common.h"

namespace arr {

namespace {

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kXcd = 8;
constexpr int64_t kRun = 32;      // consecutive rows per wave visit
constexpr int kMaxChunkLog = 5;   // at most 32 runs per XCD chunk
constexpr int kMaxGroups = 1024;  // 4 waves per SIMD on 256 CUs
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit elements

template <typename T, int V>
struct VecT {
  typedef T type __attribute__((ext_vector_type(V)));
};
template <typename T>
struct VecT<T, 1> {
  typedef T type;
};

template <int V, typename X>
__device__ __forceinline__ double lane_elem(const X &x, int v) {
  if constexpr (V == 1)
    return (double)x;
  else
    return (double)x[v];
}

template <int V, typename X, typename E>
__device__ __forceinline__ void set_elem(X &x, int v, E e) {
  if constexpr (V == 1)
    x = e;
  else
    x[v] = e;
}

// Buffer loads and stores of one lane's slot (out-of-range offsets read 0 and
// drop the store). Output rows are written once per launch: the streaming
// hint keeps them from displacing gathered rows in L2.
template <typename T, int VEC>
struct BufIO;
template <>
struct BufIO<double, 1> {
  static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  static __device__ __forceinline__ void st(double v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          off, 0, 2);
  }
};
template <>
struct BufIO<double, 2> {
  typedef double v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ v2 ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  }
  static __device__ __forceinline__ void st(v2 v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r,
                                           off, 0, 2);
  }
};
template <>
struct BufIO<float, 1> {
  static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  }
  static __device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 2);
  }
};
template <>
struct BufIO<float, 2> {
  typedef float v2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ v2 ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(v2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  }
  static __device__ __forceinline__ void st(v2 v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          off, 0, 2);
  }
};
template <>
struct BufIO<float, 4> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 ld(__amdgpu_buffer_rsrc_t r, int off) {
    return __builtin_bit_cast(v4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  }
  static __device__ __forceinline__ void st(v4 v, __amdgpu_buffer_rsrc_t r, int off) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, v), r,
                                           off, 0, 2);
  }
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, kRsrcWord3);
}

// Run assigned to the k-th slot of XCD x, chunks of 2^lg runs.
__device__ __forceinline__ int64_t xcd_run(int64_t k, int x, int lg) {
  return (((k >> lg) * kXcd + x) << lg) + (k & ((1 << lg) - 1));
}

// log2 of the chunk for w waves per XCD (w is a multiple of 4).
__device__ __forceinline__ int chunk_log(int64_t w) { return min(kMaxChunkLog, (int)__builtin_ctzll(w)); }

template <typename T>
struct RowCoef {
  T v[8];
};
struct RowCols {
  int32_t v[4];
};

template <typename T, int VEC, int NT, bool OVF, bool HASZ, bool SUMS>
__global__ __launch_bounds__(kThreads) void k_filter_spmm(
    int64_t n, const T *__restrict__ coef, const int32_t *__restrict__ fcol, const int64_t *__restrict__ orp,
    const int32_t *__restrict__ ocol, const T *__restrict__ oval, int w, const T *__restrict__ Yin, int64_t ldy,
    const T *Z, int64_t ldz, T *Yout, int64_t ldo, T alpha, T beta, T gamma, double *__restrict__ partial,
    int wtot, int c0, const double *__restrict__ colss) {
#define ARR_VBLOCK blockIdx.x
#define ARR_VGRID gridDim.x
#include "spmm_plain_body.inc"
#undef ARR_VBLOCK
#undef ARR_VGRID
}

// Paired form: a unit is an upper run [a0, a0 + kPairRun) of a block of 2P
// rows together with the lower run [a0 + P, a0 + P + kPairRun); each row's
// partner is the other run's centre row, already in registers. The runs of a
// half block start at multiples of kPairRun, except the last, which starts
// at P - kPairRun to stay inside the half: its first `skip` rows, done by the
// previous run, are computed again but neither stored (their buffer resource
// holds no records) nor summed. Rows past the last whole block take the
// guarded row-at-a-time path.
template <typename T, int VEC, int NT, int KF, bool HASZ, bool SUMS>
__global__ __launch_bounds__(kThreads) void k_filter_spmm_paired(
    int64_t n, int64_t P, const T *__restrict__ coef, const int32_t *__restrict__ fcol, int w,
    const T *__restrict__ Yin, int64_t ldy, const T *Z, int64_t ldz, T *Yout, int64_t ldo, T alpha, T beta,
    T gamma, double *__restrict__ partial, int wtot, int c0, const double *__restrict__ colss) {
#define ARR_VBLOCK blockIdx.x
#define ARR_VGRID gridDim.x
#include "spmm_paired_body.inc"
#undef ARR_VBLOCK
#undef ARR_VGRID
}

// Grid form: the operator of a 7-point stencil on a gx x gy x gz grid in
// lexicographic order (row i = (z gy + y) gx + x), or of a 5-point stencil on
// a gx x gz grid (gy = 1). Record of row i: {A[i][i - gx gy], A[i][i - gx],
// A[i][i - 1], A[i][i], A[i][i + 1], A[i][i + gx], A[i][i + gx gy], 0}, zero
// for a neighbour outside the grid (for gy = 1 the +-gx entries sit in the
// first and seventh slots).
//
// A workgroup owns an x-y tile of TX x TY grid rows, a column chunk of
// 64 VEC columns and a segment of z planes, and streams through the segment
// plane by plane (2.5D blocking). The tile's rows of plane z and their x-y
// halo sit in LDS; each thread keeps its rows of planes z - 1 and z + 1 in
// registers. Every Yin row is thus read from memory about once (plus the x-y
// halo, (2 TX + 2 TY)/(TX TY) of it, mostly an L2 hit for the neighbouring
// tiles) instead of once per stencil entry: with the store that is about 2.5
// row accesses per output row through the CU's vector memory path, against 5
// in the paired form. Wave q takes the tile rows [q R, q R + R), R = TX TY / 4;
// lane l holds columns [VEC l, VEC l + VEC) of the chunk, so one wave
// instruction moves one 512-byte row segment.
//
// Work items (segment, tile, chunk) are dealt to the XCDs in contiguous
// ranges: XCD x takes items [x I, x I + I) in order, chunks fastest, so the
// column chunks of the same rows are read at the same time (whole rows from
// each DRAM page) and a tile's x-y neighbours usually run on the same XCD at
// the same time, so its halo rows hit that XCD's L2. Column sums of squares: one partial row per
// (tile, segment), written for the chunk's columns.
constexpr int kGridWaves = 8;     // waves per workgroup of the grid form
constexpr int kGridThreads = 64 * kGridWaves;

template <int TX, int TY>
struct GridTile {
  static constexpr bool kHY = TY > 1;                       // y neighbours exist
  static constexpr int kR = TX * TY / kGridWaves;           // rows per wave
  static constexpr int kW = TX + 2;                         // LDS slots per tile row
  static constexpr int kSlots = kW * (TY + (kHY ? 2 : 0));  // tile rows plus x-y halo
  static constexpr int kHalo = 2 * TY + (kHY ? 2 * TX : 0);
  static constexpr int kHJ = (kHalo + kGridWaves - 1) / kGridWaves;  // halo rows per wave
  static_assert(TX * TY % kGridWaves == 0, "tile shape");
  static __device__ __forceinline__ int slot(int lx, int ly) { return (ly + (kHY ? 1 : 0)) * kW + lx + 1; }
  // h-th halo row of the tile: left/right columns, then (3D) bottom/top rows
  static __device__ __forceinline__ void halo(int h, int &lx, int &ly) {
    if (h < 2 * TY) {
      ly = h >> 1;
      lx = (h & 1) ? TX : -1;
    } else {
      const int g = h - 2 * TY;
      lx = g >> 1;
      ly = (g & 1) ? TY : -1;
    }
  }
};

template <typename T, int VEC, int TX, int TY, bool HASZ, bool SUMS>
__global__ __launch_bounds__(kGridThreads) void k_filter_spmm_grid(
    int gx, int gy, int gz, int ntx, int ntile, int nseg, int zlen, int nchunk, int items, int per_xcd,
    const T *__restrict__ coef, int w, const T *__restrict__ Yin, int64_t ldy, const T *Z, int64_t ldz, T *Yout,
    int64_t ldo, T alpha, T beta, T gamma, double *__restrict__ partial, int wtot, const double *__restrict__ colss) {
  typedef typename VecT<T, VEC>::type vec;
  typedef BufIO<T, VEC> IO;
  typedef GridTile<TX, TY> G;
  constexpr int R = G::kR;
  __shared__ vec L[G::kSlots][64];
  __shared__ T Kc[TX * TY][8];  // the tile rows' records of the plane in LDS
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // work item of this workgroup: XCD x = blockIdx % 8 owns a contiguous range
  const int item = (int)(blockIdx.x % kXcd) * per_xcd + (int)(blockIdx.x / kXcd);
  if (item >= items) return;  // uniform over the workgroup, before any barrier
  const int chunk = item % nchunk;
  const int tile = (item / nchunk) % ntile;
  const int seg = item / (ntile * nchunk);
  const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
  const int z0 = seg * zlen, z1 = min(gz, z0 + zlen);
  const int c0 = chunk * 64 * VEC;
  const int wc = min(64 * VEC, w - c0);
  const bool lane_in = VEC * lane < wc;  // lanes past the chunk neither store nor sum
  const int64_t plane = (int64_t)gx * gy;
  const vec zero = vec(0);
  // Rows are addressed through one buffer resource per plane and block (its
  // records end with the plane) and a byte offset that depends only on the
  // row's place in the plane, so a plane step changes one base address.
  auto in_plane = [&](int lx, int ly) -> int { return (y0 + ly) * gx + x0 + lx; };
  auto inside = [&](int lx, int ly) { return x0 + lx >= 0 && x0 + lx < gx && y0 + ly >= 0 && y0 + ly < gy; };
  // A plane's records end with the last element of this chunk in its last
  // row: lanes past the chunk may read into the next row (never stored), but
  // nothing past the caller's block.
  auto plane_rsrc = [&](const T *base, int64_t ld, int z) {
    return row_rsrc(base + (int64_t)z * plane * ld, (int)(((plane - 1) * ld + c0 + wc) * (int64_t)sizeof(T)));
  };
  const int lane_off = (c0 + VEC * lane) * (int)sizeof(T);
  auto qx = [&](int q) { return (wv * R + q) % TX; };
  auto qy = [&](int q) { return (wv * R + q) / TX; };
  uint32_t valid = 0;
#pragma unroll
  for (int q = 0; q < R; ++q) valid |= inside(qx(q), qy(q)) ? (1u << q) : 0u;
  valid = __builtin_amdgcn_readfirstlane(valid);
  auto qv = [&](int q) { return (valid >> q) & 1u; };
  vec cs = vec(1);
  if constexpr (SUMS) {
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const int c = c0 + VEC * lane + v;
      set_elem<VEC>(cs, v, (T)(colss && c < w ? 1.0 / sqrt(colss[c]) : 1.0));
    }
  }
  double ss[VEC];
#pragma unroll
  for (int v = 0; v < VEC; ++v) ss[v] = 0.0;

  // records: thread t loads value t % 8 of tile row t / 8
  static_assert(TX * TY * 8 == kGridThreads, "one record value per thread");
  const int kr = threadIdx.x >> 3, kp = threadIdx.x & 7;
  const bool kin = inside(kr % TX, kr / TX);
  const int64_t krow = in_plane(kr % TX, kr / TX);
  auto load_coef = [&](int z, T &kv) { kv = (kin && z < gz) ? coef[8 * (z * plane + krow) + kp] : T(0); };

  auto load_rows = [&](int z, vec *dst) {
    if (z < 0 || z >= gz) {
#pragma unroll
      for (int q = 0; q < R; ++q) dst[q] = zero;
      return;
    }
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(Yin, ldy, z);
#pragma unroll
    for (int q = 0; q < R; ++q)
      dst[q] = qv(q) ? IO::ld(r, (int)(in_plane(qx(q), qy(q)) * ldy * (int64_t)sizeof(T)) + lane_off) : zero;
  };
  auto load_halo = [&](int z, vec *dst) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(Yin, ldy, z);
#pragma unroll
    for (int j = 0; j < G::kHJ; ++j) {
      const int h = wv + kGridWaves * j;
      int lx = 0, ly = 0;
      if (h < G::kHalo) G::halo(h, lx, ly);
      dst[j] = (h < G::kHalo && inside(lx, ly))
                   ? IO::ld(r, (int)(in_plane(lx, ly) * ldy * (int64_t)sizeof(T)) + lane_off)
                   : zero;
    }
  };
  auto store_plane = [&](const vec *rows, const vec *hal) {
#pragma unroll
    for (int q = 0; q < R; ++q) L[G::slot(qx(q), qy(q))][lane] = rows[q];
#pragma unroll
    for (int j = 0; j < G::kHJ; ++j) {
      const int h = wv + kGridWaves * j;
      if (h < G::kHalo) {
        int lx, ly;
        G::halo(h, lx, ly);
        L[G::slot(lx, ly)][lane] = hal[j];
      }
    }
  };

  // Four register sets hold this wave's rows of planes z - 1, z, z + 1 and
  // z + 2 at step z and rotate roles from step to step; two sets of halo
  // rows and records (planes z + 1 and z + 2) alternate. Loads for plane
  // z + 2 are issued a whole step before their use, and no register is copied
  // to another (a copy would wait for its load).
  vec S0[R], S1[R], S2[R], S3[R], HA[G::kHJ], HB[G::kHJ];
  T KA, KB;
  auto step = [&](int z, const vec *Pv, const vec *C, const vec *Nv, vec *N2, const vec *Hn, vec *Hn2, const T &Kn,
                  T &Kn2) {
    const bool more = z + 1 < z1;
    if (more) load_rows(z + 2, N2);
    if (z + 2 < z1) {
      load_halo(z + 2, Hn2);
      load_coef(z + 2, Kn2);
    }
    const __amdgpu_buffer_rsrc_t ro = plane_rsrc(Yout, ldo, z);
    const __amdgpu_buffer_rsrc_t rz = plane_rsrc(HASZ ? Z : Yout, HASZ ? ldz : ldo, z);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      if (!qv(q)) continue;  // wave-uniform
      const int lx = qx(q), ly = qy(q);
      const T *k = Kc[wv * R + q];
      vec acc = k[3] * C[q];
      acc += k[2] * L[G::slot(lx - 1, ly)][lane];
      acc += k[4] * L[G::slot(lx + 1, ly)][lane];
      if constexpr (G::kHY) {
        acc += k[1] * L[G::slot(lx, ly - 1)][lane];
        acc += k[5] * L[G::slot(lx, ly + 1)][lane];
      }
      acc += k[0] * Pv[q];
      acc += k[6] * Nv[q];
      vec o = alpha * acc;
      if (beta != T(0)) o += beta * C[q];
      const int row = in_plane(lx, ly);
      if constexpr (HASZ) o += gamma * IO::ld(rz, (int)(row * ldz * (int64_t)sizeof(T)) + lane_off);
      if constexpr (SUMS) o *= cs;
      if (lane_in) IO::st(o, ro, (int)(row * ldo * (int64_t)sizeof(T)) + lane_off);
      if constexpr (SUMS) {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
          const double ov = lane_in ? lane_elem<VEC>(o, v) : 0.0;
          ss[v] = fma(ov, ov, ss[v]);
        }
      }
    }
    if (more) {
      __syncthreads();  // every wave is done with plane z in LDS
      store_plane(Nv, Hn);
      Kc[kr][kp] = Kn;
      __syncthreads();
    }
  };

  // prologue: plane z0 into LDS and S1, z0 - 1 in S0, z0 + 1 in S2 (with its
  // halo and records in HA, KA)
  load_rows(z0 - 1, S0);
  load_rows(z0, S1);
  load_halo(z0, HA);
  load_coef(z0, KA);
  store_plane(S1, HA);
  Kc[kr][kp] = KA;
  load_rows(z0 + 1, S2);
  if (z0 + 1 < z1) {
    load_halo(z0 + 1, HA);
    load_coef(z0 + 1, KA);
  }
  __syncthreads();
  for (int z = z0; z < z1; z += 4) {
    step(z, S0, S1, S2, S3, HA, HB, KA, KB);
    if (z + 1 < z1) step(z + 1, S1, S2, S3, S0, HB, HA, KB, KA);
    if (z + 2 < z1) step(z + 2, S2, S3, S0, S1, HA, HB, KA, KB);
    if (z + 3 < z1) step(z + 3, S3, S0, S1, S2, HB, HA, KB, KA);
  }

  if constexpr (SUMS) {
    __syncthreads();  // the plane buffer is reused for the reduction
    double *red = reinterpret_cast<double *>(&L[0][0]);
#pragma unroll
    for (int v = 0; v < VEC; ++v) red[wv * 64 * VEC + VEC * lane + v] = ss[v];
    __syncthreads();
    for (int c = threadIdx.x; c < wc; c += kGridThreads) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < kGridWaves; ++q) sum += red[q * 64 * VEC + c];
      partial[(int64_t)(tile * nseg + seg) * wtot + c0 + c] = sum;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_spmv_grid(int64_t n, int64_t gx, int64_t gy, const T *__restrict__ coef,
                                                   const T *__restrict__ x, T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T *k = coef + 8 * i;
  const int64_t plane = gx * gy;
  T s = k[3] * x[i];
  if (k[2] != T(0)) s = fma(k[2], x[i - 1], s);
  if (k[4] != T(0)) s = fma(k[4], x[i + 1], s);
  if (k[1] != T(0)) s = fma(k[1], x[i - gx], s);
  if (k[5] != T(0)) s = fma(k[5], x[i + gx], s);
  if (k[0] != T(0)) s = fma(k[0], x[i - plane], s);
  if (k[6] != T(0)) s = fma(k[6], x[i + plane], s);
  y[i] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_spmv(int64_t n, int64_t P, const T *__restrict__ coef,
                                              const int32_t *__restrict__ fcol, const int64_t *__restrict__ orp,
                                              const int32_t *__restrict__ ocol, const T *__restrict__ oval,
                                              const T *__restrict__ x, T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T *k = coef + 8 * i;
  T s = k[1] * x[i];
  if (i > 0) s = fma(k[0], x[i - 1], s);
  if (i + 1 < n) s = fma(k[2], x[i + 1], s);
  for (int e = 0; e < 4; ++e) s = fma(k[3 + e], x[fcol[4 * i + e]], s);
  if (P) {
    const int64_t pi = (i % (2 * P)) < P ? i + P : i - P;
    if (pi < n) s = fma(k[7], x[pi], s);
  }
  if (orp)
    for (int64_t p = orp[i]; p < orp[i + 1]; ++p) s = fma(oval[p], x[ocol[p]], s);
  y[i] = s;
}

// Multi-request kernel: workgroup g runs tasks g, g + gridDim.x, ... of the
// table; each task is one workgroup of the collected launch desc[task.x]
// (FORM 0: plain form, X = overflow rows; FORM 1: paired form, X = far
// slots), run by the same body as that launch's own kernel.
template <typename T, int VEC, int NT, int FORM, int X, bool HASZ, bool SUMS>
__global__ __launch_bounds__(kThreads) void k_filter_spmm_tasks(const SpmmTask *__restrict__ desc,
                                                                const int2 *__restrict__ tasks, int ntasks) {
  for (int task = blockIdx.x; task < ntasks; task += gridDim.x) {
    const int2 tk = tasks[task];
    const SpmmTask &d = desc[tk.x];
    const unsigned vblock = (unsigned)tk.y, vgrid = (unsigned)d.groups;
    int64_t n = d.n, ldy = d.ldy, ldz = d.ldz, ldo = d.ldo;
    const T *coef = (const T *)d.coef;
    const int32_t *fcol = d.fcol;
    const T *Yin = (const T *)d.Yin, *Z = (const T *)d.Z;
    T *Yout = (T *)d.Yout;
    T alpha = (T)d.alpha, beta = (T)d.beta, gamma = (T)d.gamma;
    double *partial = d.partial;
    const double *colss = d.colss;
    int w = d.w, wtot = d.wtot, c0 = d.c0;
#define ARR_VBLOCK vblock
#define ARR_VGRID vgrid
    if constexpr (FORM == 0) {
      constexpr bool OVF = X != 0;
      const int64_t *orp = d.orp;
      const int32_t *ocol = d.ocol;
      const T *oval = (const T *)d.oval;
#include "spmm_plain_body.inc"
    } else {
      constexpr int KF = X;
      int64_t P = d.P;
#include "spmm_paired_body.inc"
    }
#undef ARR_VBLOCK
#undef ARR_VGRID
    __syncthreads();  // the column-sum reduction's LDS is reused by the next task
  }
}

template <typename T, int VEC, int NT, int FORM, int X, bool HASZ, bool SUMS>
void launch_tasks(const SpmmTask *desc, const int2 *tasks, int ntasks, hipStream_t s) {
  const int grid = std::min(ntasks, kMaxGroups);
  hipLaunchKernelGGL((k_filter_spmm_tasks<T, VEC, NT, FORM, X, HASZ, SUMS>), dim3(grid), dim3(kThreads), 0, s, desc,
                     tasks, ntasks);
}

template <typename T, int VEC, int NT, bool OVF, bool HASZ, bool SUMS>
void launch_variant(const DevCSR<T> &A, Blk<const T> Yin, const T *zp, int64_t ldz, Blk<T> Yout, int w, int c0,
                    T alpha, T beta, T gamma, double *partial, int wtot, int groups, const double *colss,
                    hipStream_t s) {
  if (SpmmBatch *b = spmm_batch()) {
    b->add(SpmmTask{A.n, 0, Yin.ld, ldz, Yout.ld, A.coef, A.fcol, A.orp, A.ocol, A.oval, Yin.p + c0, zp,
                    Yout.p + c0, (double)alpha, (double)beta, (double)gamma, partial, colss ? colss + c0 : nullptr, w,
                    wtot, c0, groups},
           &launch_tasks<T, VEC, NT, 0, OVF ? 1 : 0, HASZ, SUMS>);
    return;
  }
  hipLaunchKernelGGL((k_filter_spmm<T, VEC, NT, OVF, HASZ, SUMS>), dim3(groups), dim3(kThreads), 0, s, A.n, A.coef,
                     A.fcol, A.orp, A.ocol, A.oval, w, Yin.p + c0, Yin.ld, zp, ldz, Yout.p + c0, Yout.ld, alpha, beta,
                     gamma, partial, wtot, c0, colss ? colss + c0 : nullptr);
}

template <typename T, int VEC, int NT>
void launch_nt(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, int w, int c0, T alpha,
               T beta, T gamma, double *partial, int wtot, int groups, const double *colss, hipStream_t s) {
  const T *zp = Z.p ? Z.p + c0 : nullptr;
  const int sel = (A.orp ? 4 : 0) + (zp ? 2 : 0) + (partial ? 1 : 0);
#define ARR_SPMM_CASE(k, O, H, S)                                                                        \
  case k:                                                                                               \
    launch_variant<T, VEC, NT, O, H, S>(A, Yin, zp, Z.ld, Yout, w, c0, alpha, beta, gamma, partial, wtot, \
                                        groups, colss, s);                                              \
    break;
  switch (sel) {
    ARR_SPMM_CASE(0, false, false, false)
    ARR_SPMM_CASE(1, false, false, true)
    ARR_SPMM_CASE(2, false, true, false)
    ARR_SPMM_CASE(3, false, true, true)
    ARR_SPMM_CASE(4, true, false, false)
    ARR_SPMM_CASE(5, true, false, true)
    ARR_SPMM_CASE(6, true, true, false)
    ARR_SPMM_CASE(7, true, true, true)
  }
#undef ARR_SPMM_CASE
}

template <typename T, int VEC, int NT, int KF, bool HASZ, bool SUMS>
void launch_paired_variant(const DevCSR<T> &A, Blk<const T> Yin, const T *zp, int64_t ldz, Blk<T> Yout, int w, int c0,
                           T alpha, T beta, T gamma, double *partial, int wtot, int groups, const double *colss,
                           hipStream_t s) {
  if (SpmmBatch *b = spmm_batch()) {
    b->add(SpmmTask{A.n, A.pair, Yin.ld, ldz, Yout.ld, A.coef, A.fcol, nullptr, nullptr, nullptr, Yin.p + c0, zp,
                    Yout.p + c0, (double)alpha, (double)beta, (double)gamma, partial, colss ? colss + c0 : nullptr, w,
                    wtot, c0, groups},
           &launch_tasks<T, VEC, NT, 1, KF, HASZ, SUMS>);
    return;
  }
  hipLaunchKernelGGL((k_filter_spmm_paired<T, VEC, NT, KF, HASZ, SUMS>), dim3(groups), dim3(kThreads), 0, s, A.n,
                     A.pair, A.coef, A.fcol, w, Yin.p + c0, Yin.ld, zp, ldz, Yout.p + c0, Yout.ld, alpha, beta, gamma,
                     partial, wtot, c0, colss ? colss + c0 : nullptr);
}

template <typename T, int VEC, int NT>
void launch_paired_nt(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, int w, int c0, T alpha,
                      T beta, T gamma, double *partial, int wtot, int groups, const double *colss,
                      hipStream_t s) {
  const T *zp = Z.p ? Z.p + c0 : nullptr;
  const int sel = (A.kf == 1 ? 4 : 0) + (zp ? 2 : 0) + (partial ? 1 : 0);
#define ARR_SPMM_CASE(k, KF, H, S)                                                                              \
  case k:                                                                                                      \
    launch_paired_variant<T, VEC, NT, KF, H, S>(A, Yin, zp, Z.ld, Yout, w, c0, alpha, beta, gamma, partial, wtot, \
                                                groups, colss, s);                                             \
    break;
  switch (sel) {
    ARR_SPMM_CASE(0, 3, false, false)
    ARR_SPMM_CASE(1, 3, false, true)
    ARR_SPMM_CASE(2, 3, true, false)
    ARR_SPMM_CASE(3, 3, true, true)
    ARR_SPMM_CASE(4, 1, false, false)
    ARR_SPMM_CASE(5, 1, false, true)
    ARR_SPMM_CASE(6, 1, true, false)
    ARR_SPMM_CASE(7, 1, true, true)
  }
#undef ARR_SPMM_CASE
}

// Either form's kernel for one column chunk.
template <typename T, int VEC, int NT>
void launch_form(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, int w, int c0, T alpha,
                 T beta, T gamma, double *partial, int wtot, int groups, const double *colss, hipStream_t s) {
  if (A.pair)
    launch_paired_nt<T, VEC, NT>(A, Yin, Z, Yout, w, c0, alpha, beta, gamma, partial, wtot, groups, colss, s);
  else
    launch_nt<T, VEC, NT>(A, Yin, Z, Yout, w, c0, alpha, beta, gamma, partial, wtot, groups, colss, s);
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Work decomposition of the grid form for a block of w columns.
struct GridPlan {
  int tx, ty, vec, ntx, ntile, nchunk, nseg, zlen, items, per_xcd;
};
constexpr int kGridTargetItems = 3072;  // about four rounds of 3 workgroups on each of 256 CUs
constexpr int kGridMinZlen = 8;         // planes per segment: bounds the z halo re-read to 1/4

GridPlan grid_plan(int64_t gx, int64_t gy, int64_t gz, int w, int vec, int max_slots) {
  GridPlan p;
  p.tx = gy > 1 ? 8 : 64;
  p.ty = gy > 1 ? 8 : 1;
  p.vec = vec;
  p.ntx = (int)((gx + p.tx - 1) / p.tx);
  p.ntile = p.ntx * (int)((gy + p.ty - 1) / p.ty);
  p.nchunk = (w + 64 * vec - 1) / (64 * vec);
  const int64_t base = (int64_t)p.ntile * p.nchunk;
  int64_t nseg = (kGridTargetItems + base - 1) / base;
  nseg = std::min<int64_t>(nseg, std::max<int64_t>(1, gz / kGridMinZlen));
  // one partial row of column sums per (tile, segment)
  nseg = std::max<int64_t>(1, std::min<int64_t>(nseg, max_slots / p.ntile));
  p.zlen = (int)((gz + nseg - 1) / nseg);
  p.nseg = (int)((gz + p.zlen - 1) / p.zlen);
  p.items = (int)(base * p.nseg);
  p.per_xcd = (p.items + kXcd - 1) / kXcd;
  return p;
}

template <typename T, int VEC, int TX, int TY>
void launch_grid_tile(const DevCSR<T> &A, const GridPlan &p, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, int w,
                      T alpha, T beta, T gamma, double *partial, const double *colss, hipStream_t s) {
  const int sel = (Z.p ? 2 : 0) + (partial ? 1 : 0);
  const dim3 grid((unsigned)(p.per_xcd * kXcd)), block(kGridThreads);
#define ARR_GRID_CASE(k, H, S)                                                                                  \
  case k:                                                                                                      \
    hipLaunchKernelGGL((k_filter_spmm_grid<T, VEC, TX, TY, H, S>), grid, block, 0, s, (int)A.gx, (int)A.gy,     \
                       (int)A.gz, p.ntx, p.ntile, p.nseg, p.zlen, p.nchunk, p.items, p.per_xcd, A.coef, w, Yin.p, \
                       Yin.ld, Z.p, Z.ld, Yout.p, Yout.ld, alpha, beta, gamma, partial, w, colss);             \
    break;
  switch (sel) {
    ARR_GRID_CASE(0, false, false)
    ARR_GRID_CASE(1, false, true)
    ARR_GRID_CASE(2, true, false)
    ARR_GRID_CASE(3, true, true)
  }
#undef ARR_GRID_CASE
}

template <typename T, int VEC>
void launch_grid_vec(const DevCSR<T> &A, const GridPlan &p, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, int w,
                     T alpha, T beta, T gamma, double *partial, const double *colss, hipStream_t s) {
  if (p.ty > 1)
    launch_grid_tile<T, VEC, 8, 8>(A, p, Yin, Z, Yout, w, alpha, beta, gamma, partial, colss, s);
  else
    launch_grid_tile<T, VEC, 64, 1>(A, p, Yin, Z, Yout, w, alpha, beta, gamma, partial, colss, s);
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7) == 0; }

}  // namespace

SpmmTimer *&spmm_timer() {
  static thread_local SpmmTimer *t = nullptr;
  return t;
}

SpmmTimer *&gemm_timer() {
  static thread_local SpmmTimer *t = nullptr;
  return t;
}

SpmmTimer::Scope::Scope(SpmmTimer *t_, int cls, double work, hipStream_t s_) : t(t_), s(s_) {
  if (!t) return;
  p.a = t->get();
  p.b = t->get();
  p.cls = cls;
  p.bytes = work;
  ARR_HIP(hipEventRecord(p.a, s));
}

SpmmTimer::Scope::~Scope() {
  if (!t) return;
  // a launch that failed leaves the pair unrecorded: it is returned unused
  if (hipEventRecord(p.b, s) == hipSuccess && !std::uncaught_exceptions()) {
    try {
      t->pending.push_back(p);
      return;
    } catch (...) {
    }
  }
  t->pool.push_back(p.a);
  t->pool.push_back(p.b);
}

hipEvent_t SpmmTimer::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  ARR_HIP(hipEventCreate(&e));
  return e;
}

void SpmmTimer::flush() {
  for (Pending &p : pending) {
    ARR_HIP(hipEventSynchronize(p.b));
    float t = 0.f;
    ARR_HIP(hipEventElapsedTime(&t, p.a, p.b));
    launches[p.cls] += 1;
    ms[p.cls] += t;
    bytes[p.cls] += p.bytes;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void SpmmTimer::reset() {
  flush();
  for (int i = 0; i < kClasses; ++i) launches[i] = 0, ms[i] = 0, bytes[i] = 0;
}

SpmmTimer::~SpmmTimer() {
  for (Pending &p : pending) pool.push_back(p.a), pool.push_back(p.b);
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

int spmm_groups(int64_t n) {
  // one wave per run, at most kMaxGroups workgroups; a multiple of the XCD count
  const int64_t runs = (n + kRun - 1) / kRun;
  int64_t g = std::min<int64_t>((runs + kWaves - 1) / kWaves, kMaxGroups);
  g = std::max<int64_t>(kXcd, (g + kXcd - 1) / kXcd * kXcd);
  return (int)g;
}

namespace {

bool has_entry(const int64_t *rowptr, const int32_t *col, int64_t i, int64_t j) {
  const int32_t *b = col + rowptr[i], *e = col + rowptr[i + 1];
  const int32_t *f = std::lower_bound(b, e, (int32_t)j);
  return f != e && *f == j;
}

// Pairing offset of the paired form, or 0: candidates are the offsets
// d = j - i >= kPairRun seen in at least a quarter of a sample of rows; each
// is then counted exactly. Ties keep the smaller offset.
int64_t choose_pair(int64_t n, const int64_t *rowptr, const int32_t *col) {
  if (n < 2 * kPairRun) return 0;
  std::map<int64_t, int64_t> seen;
  const int64_t ns = std::min<int64_t>(n, 1024);
  for (int64_t t = 0; t < ns; ++t) {
    const int64_t i = t * n / ns;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
      if (col[q] - i >= kPairRun) ++seen[col[q] - i];
  }
  int64_t best = 0, best_count = 0;
  for (const auto &dc : seen) {
    const int64_t d = dc.first;
    const int64_t half_runs = (d + kPairRun - 1) / kPairRun;
    if (4 * dc.second < ns || 2 * d > n || 8 * (half_runs * kPairRun - d) > d) continue;
    int64_t c = 0;
    for (int64_t i = 0; i + d < n; ++i) c += has_entry(rowptr, col, i, i + d);
    if (2 * c >= n && c > best_count) best = d, best_count = c;
  }
  return best;
}

// One row of either form; false if a paired row has more than three far
// entries besides its partner.
bool split_row(int64_t i, int64_t P, const int64_t *rowptr, const int32_t *col, const double *val, RowSplit &out,
               int &far_max) {
  const int64_t partner = P == 0 ? -1 : (i % (2 * P)) < P ? i + P : i - P;
  const int slots = P == 0 ? 4 : 3;
  int slot = 0;
  for (int e = 0; e < 4; ++e) out.fcol[4 * i + e] = (int32_t)i;  // padding: column i, value 0
  for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
    const int64_t j = col[q];
    if (j == i - 1)
      out.coef[8 * i] = val[q];
    else if (j == i)
      out.coef[8 * i + 1] = val[q];
    else if (j == i + 1)
      out.coef[8 * i + 2] = val[q];
    else if (j == partner)
      out.coef[8 * i + 7] = val[q];
    else if (slot < slots) {
      out.fcol[4 * i + slot] = (int32_t)j;
      out.coef[8 * i + 3 + slot] = val[q];
      ++slot;
    } else if (P == 0) {
      out.ocol.push_back((int32_t)j);
      out.oval.push_back(val[q]);
    } else {
      return false;
    }
  }
  far_max = std::max(far_max, slot);
  return true;
}

// Grid form: (gx, gy, gz) when every entry of the pattern is a neighbour of
// its row in a 7-point stencil on a gx x gy x gz lexicographic grid (x
// fastest), or in a 5-point stencil on a gx x gz grid (returned with gy = 1).
// The strides are the positive column offsets above 1: exactly two, s2 < s3
// with s3 = s2 gy and n = s3 gz (3D), or one, s2 = gx with n = gx gz (2D).
// Every entry is then checked to stay inside the grid (no wrap-around from one
// grid line to the next). The tiles of the kernel must fit the rows of column
// sums (one per tile and segment).
bool choose_grid(int64_t n, const int64_t *rowptr, const int32_t *col, int64_t &gx, int64_t &gy, int64_t &gz) {
  gx = gy = gz = 0;
  if (n < 4) return false;
  int64_t s2 = 0, s3 = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      const int64_t d = (int64_t)col[q] - i;
      if (d <= 1 || d == s2 || d == s3) continue;
      if (!s2) s2 = d;
      else if (!s3) s3 = d;
      else return false;  // a third stride
    }
  if (!s2) return false;
  if (s3 && s3 < s2) std::swap(s2, s3);
  int64_t X, Y, Zd;
  if (s3) {
    if (s3 % s2 || n % s3) return false;
    X = s2, Y = s3 / s2, Zd = n / s3;
  } else {
    if (n % s2) return false;
    X = s2, Y = 1, Zd = n / s2;
  }
  if (X < 2 || Zd < 2 || (s3 && Y < 2)) return false;
  const int64_t plane = X * Y;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t x = i % X, y = (i / X) % Y, z = i / plane;
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      const int64_t d = (int64_t)col[q] - i;
      bool ok;
      if (d == 0) ok = true;
      else if (d == 1 || d == -1) ok = x + d >= 0 && x + d < X;
      else if (Y > 1 && (d == X || d == -X)) ok = y + d / X >= 0 && y + d / X < Y;
      else if (d == plane || d == -plane) ok = z + d / plane >= 0 && z + d / plane < Zd;
      else ok = false;
      if (!ok) return false;
    }
  }
  // tiles of the kernel (8 x 8 in 3D, 64 x 1 in 2D) against the column-sum rows
  const int64_t tiles = Y > 1 ? ((X + 7) / 8) * ((Y + 7) / 8) : (X + 63) / 64;
  if (tiles > spmm_groups(n) || n > (int64_t)INT32_MAX) return false;
  gx = X, gy = Y, gz = Zd;
  return true;
}

// Rows in the grid form's record: {A[i][i - gx gy], A[i][i - gx], A[i][i - 1],
// A[i][i], A[i][i + 1], A[i][i + gx], A[i][i + gx gy], 0}.
void split_grid(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, RowSplit &out) {
  const int64_t plane = out.gx * out.gy;
  out.coef.assign(8 * n, 0.0);
  out.fcol.clear();
  out.orp.clear();
  out.ocol.clear();
  out.oval.clear();
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      const int64_t d = (int64_t)col[q] - i;
      const int slot = d == 0 ? 3 : d == -1 ? 2 : d == 1 ? 4 : d == -plane ? 0 : d == plane ? 6 : d < 0 ? 1 : 5;
      out.coef[8 * i + slot] = val[q];
    }
  out.pair = 0;
  out.kf = 0;
}

}  // namespace

void split_rows(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, RowSplit &out,
                int form) {
  // automatic: the grid form for 2D grids only (measured faster than the
  // paired form there; slower on 3D grids, where it is taken only on request)
  const bool allow_grid = form == 0 || form == 3, allow_pair = form != 1;
  if (allow_grid && choose_grid(n, rowptr, col, out.gx, out.gy, out.gz) && (form == 3 || out.gy == 1)) {
    split_grid(n, rowptr, col, val, out);
    return;
  }
  out.gx = out.gy = out.gz = 0;
  int64_t P = allow_pair ? choose_pair(n, rowptr, col) : 0;
  for (;;) {
    out.coef.assign(8 * n, 0.0);
    out.fcol.assign(4 * n, 0);
    out.orp.assign(n + 1, 0);
    out.ocol.clear();
    out.oval.clear();
    int far_max = 0;
    bool fits = true;
    for (int64_t i = 0; i < n && fits; ++i) {
      fits = split_row(i, P, rowptr, col, val, out, far_max);
      out.orp[i + 1] = (int64_t)out.ocol.size();
    }
    if (!fits) {
      P = 0;  // a row too long for the paired form: plain form
      continue;
    }
    out.pair = P;
    out.kf = P == 0 ? 4 : far_max <= 1 ? 1 : 3;
    break;
  }
  if (out.ocol.empty()) out.orp.clear();
}

// Grid form: FP32 rows with 8-byte alignment take two columns per lane
// (512-byte segments).
template <typename T>
bool grid_vec2(Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout) {
  const int w = Yout.w;
  return sizeof(T) == 4 && w % 2 == 0 && Yin.ld % 2 == 0 && Yout.ld % 2 == 0 && (!Z.p || Z.ld % 2 == 0) &&
         aligned8(Yin.p) && aligned8(Yout.p) && (!Z.p || aligned8(Z.p));
}

// What launch_filter_spmm returns for these arguments (the rows of column
// partial sums its launches write), without launching anything.
template <typename T>
int filter_spmm_groups(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout) {
  const int groups = spmm_groups(A.n);
  if (!A.gx || A.n == 0 || Yout.w == 0) return groups;
  const GridPlan p = grid_plan(A.gx, A.gy, A.gz, Yout.w, grid_vec2<T>(Yin, Z, Yout) ? 2 : 1, groups);
  return p.ntile * p.nseg;
}

template <typename T>
int launch_filter_spmm(const DevCSR<T> &A, Blk<const T> Yin, Blk<const T> Z, Blk<T> Yout, double alpha,
                       double beta, double gamma, double *partial, hipStream_t s, const double *colss) {
  const int w = Yout.w;
  ARR_REQUIRE(Yin.w >= w && (!Z.p || Z.w >= w), "filter_spmm: block widths differ");
  ARR_REQUIRE(Yin.p != Yout.p, "filter_spmm: Yout must not alias Yin");
  ARR_REQUIRE(!colss || partial, "filter_spmm: output column scaling needs the column sums");
  ARR_REQUIRE(A.n == 0 || (A.coef && (A.fcol || A.gx)), "filter_spmm: matrix rows missing");
  ARR_REQUIRE(!A.orp || (A.ocol && A.oval), "filter_spmm: overflow entries missing");
  ARR_REQUIRE(A.pair == 0 || (!A.orp && A.pair >= kPairRun && 2 * A.pair <= A.n && (A.kf == 1 || A.kf == 3)),
              "filter_spmm: invalid paired form");
  if (SpmmSink *k = spmm_sink()) {
    // A outlives the call (the solver's matrix); the rest is copied
    k->run([=, &A](hipStream_t bs) { launch_filter_spmm<T>(A, Yin, Z, Yout, alpha, beta, gamma, partial, bs, colss); },
           s);
    return filter_spmm_groups<T>(A, Yin, Z, Yout);
  }
  const int groups = spmm_groups(A.n);
  if (A.n == 0 || w == 0) return groups;
  SpmmTimer *timer = spmm_batch() ? nullptr : spmm_timer();  // collected launches are not timed
  if (A.gx) {
    ARR_REQUIRE(A.gx * A.gy * A.gz == A.n && A.pair == 0 && !A.orp, "filter_spmm: invalid grid form");
    const bool v2 = grid_vec2<T>(Yin, Z, Yout);
    const int vec = v2 ? 2 : 1;
    const GridPlan p = grid_plan(A.gx, A.gy, A.gz, w, vec, groups);
    // rows are addressed by 32-bit byte offsets within a plane of each block
    const int64_t plane = A.gx * A.gy, lmax = std::max(Yin.ld, std::max(Yout.ld, Z.p ? Z.ld : (int64_t)0));
    ARR_REQUIRE(plane * (lmax + 64 * vec) * (int64_t)sizeof(T) <= (int64_t)INT32_MAX,
                "filter_spmm: grid plane too large for the block's leading dimension");
    ARR_REQUIRE(!partial || p.ntile * p.nseg <= groups, "filter_spmm: grid tiles exceed the column-sum rows");
    const int flags = (Z.p ? 1 : 0) + (partial ? 4 : 0) + 32 + (p.ty == 1 ? 64 : 0);
    const int cls = (vec == 2 ? 1 : 0) + (sizeof(T) == 8 ? 10 : 0) + 20 * flags;
    SpmmTimer::Pending pend{};
    if (timer) {
      pend.a = timer->get();
      pend.b = timer->get();
      pend.cls = cls;
      pend.bytes = (double)(sizeof(T) + 4) * A.nnz + 8.0 * (A.n + 1) +
                   (double)sizeof(T) * A.n * w * (2.0 + (Z.p ? 1.0 : 0.0));
      ARR_HIP(hipEventRecord(pend.a, s));
    }
    const T al = (T)alpha, be = (T)beta, ga = (T)gamma;
    if (v2) {
      if constexpr (sizeof(T) == 4) launch_grid_vec<T, 2>(A, p, Yin, Z, Yout, w, al, be, ga, partial, colss, s);
    } else {
      launch_grid_vec<T, 1>(A, p, Yin, Z, Yout, w, al, be, ga, partial, colss, s);
    }
    ARR_HIP(hipGetLastError());
    if (timer) {
      ARR_HIP(hipEventRecord(pend.b, s));
      timer->pending.push_back(pend);
    }
    return p.ntile * p.nseg;
  }
  // FP32 with 16-byte aligned rows: 4 consecutive columns per lane
  const bool vec4 = sizeof(T) == 4 && Yin.ld % 4 == 0 && Yout.ld % 4 == 0 && (!Z.p || Z.ld % 4 == 0) &&
                    aligned16(Yin.p) && aligned16(Yout.p) && (!Z.p || aligned16(Z.p)) && w % 4 == 0;
  // Column chunks: at most 4 slots per lane for FP64 (256 columns), 2 with
  // 16-byte FP32 loads (512 columns), 1 for FP32 rows that are not 16-byte
  // aligned (64 columns)
  // FP64 in the paired form with 16-byte aligned rows and an even width: two
  // consecutive columns per lane (128 columns per wave instruction); the
  // plain form keeps 8-byte loads, which measured faster there
  const bool vec2 = sizeof(T) == 8 && A.pair && Yin.ld % 2 == 0 && Yout.ld % 2 == 0 &&
                    (!Z.p || Z.ld % 2 == 0) && aligned16(Yin.p) && aligned16(Yout.p) && (!Z.p || aligned16(Z.p)) &&
                    w % 2 == 0;
  const int chunk = vec4 ? 512 : sizeof(T) == 8 ? 256 : 64;
  for (int c0 = 0; c0 < w; c0 += chunk) {
    const int wc = std::min(chunk, w - c0);
    const T al = (T)alpha, be = (T)beta, ga = (T)gamma;
    const int slots = vec4   ? 4 * ((wc + 255) / 256)
                      : vec2 ? 2 * ((wc + 127) / 128)
                             : (wc + 63) / 64;  // columns per lane
    const int flags = (Z.p ? 1 : 0) + (A.orp ? 2 : 0) + (partial ? 4 : 0) + (A.pair ? 8 : 0) +
                      (A.pair && A.kf == 1 ? 16 : 0);
    const int cls = (slots <= 1 ? 0 : slots <= 2 ? 1 : slots <= 4 ? 2 : slots <= 8 ? 3 : 4) +
                    (vec4 || vec2 ? 5 : 0) + (sizeof(T) == 8 ? 10 : 0) + 20 * flags;
    SpmmTimer::Pending pend{};
    if (timer) {
      pend.a = timer->get();
      pend.b = timer->get();
      pend.cls = cls;
      // algorithmic bytes: the matrix once (CSR of all its entries), gathered
      // Yin once, Z, Yout
      pend.bytes = (double)(sizeof(T) + 4) * A.nnz + 8.0 * (A.n + 1) +
                   (double)sizeof(T) * A.n * wc * (2.0 + (Z.p ? 1.0 : 0.0));
      ARR_HIP(hipEventRecord(pend.a, s));
    }
    if (vec4) {
      if constexpr (sizeof(T) == 4) {
        if (wc <= 256)
          launch_form<T, 4, 1>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, colss, s);
        else
          launch_form<T, 4, 2>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, colss, s);
      }
    } else if (vec2) {
      if constexpr (sizeof(T) == 8) {
        if (wc <= 128)
          launch_paired_nt<T, 2, 1>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, colss, s);
        else
          launch_paired_nt<T, 2, 2>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, colss, s);
      }
    } else if (wc <= 64) {
      launch_form<T, 1, 1>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, colss, s);
    } else if constexpr (sizeof(T) == 8) {
      if (wc <= 128)
        launch_form<T, 1, 2>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, colss, s);
      else
        launch_form<T, 1, 4>(A, Yin, Z, Yout, wc, c0, al, be, ga, partial, w, groups, colss, s);
    }
    if (timer) {
      ARR_HIP(hipEventRecord(pend.b, s));
      timer->pending.push_back(pend);
    }
  }
  ARR_HIP(hipGetLastError());
  return groups;
}

template <typename T>
void launch_spmv(const DevCSR<T> &A, const T *x, T *y, hipStream_t s) {
  if (A.n == 0) return;
  const int64_t blocks = (A.n + 255) / 256;
  if (A.gx)
    hipLaunchKernelGGL((k_spmv_grid<T>), dim3((unsigned)blocks), dim3(256), 0, s, A.n, A.gx, A.gy, A.coef, x, y);
  else
    hipLaunchKernelGGL((k_spmv<T>), dim3((unsigned)blocks), dim3(256), 0, s, A.n, A.pair, A.coef, A.fcol, A.orp,
                       A.ocol, A.oval, x, y);
  ARR_HIP(hipGetLastError());
}

template int launch_filter_spmm<double>(const DevCSR<double> &, Blk<const double>, Blk<const double>,
                                        Blk<double>, double, double, double, double *, hipStream_t,
                                        const double *);
template int launch_filter_spmm<float>(const DevCSR<float> &, Blk<const float>, Blk<const float>, Blk<float>,
                                       double, double, double, double *, hipStream_t, const double *);
template void launch_spmv<double>(const DevCSR<double> &, const double *, double *, hipStream_t);
template void launch_spmv<float>(const DevCSR<float> &, const float *, float *, hipStream_t);

}  // namespace arr
