// bfloat16 NMF pass over p on the matrix cores (eq. 4), float32 accumulation.
//
// One persistent 512-thread workgroup per CU walks tiles of 16 rows of the
// bfloat16 copy of p (row pitch ldb, zero-padded to a multiple of 32 bins).
// Wave w owns a contiguous range of 32-bin k-steps for the whole pass.  Per
// tile:
//   1. the wave writes its bins of the 16 rows (loaded coalesced, 1 KB per
//      instruction, prefetched two tiles ahead) into a row-major LDS tile;
//   2. N_V = P D on MFMA 16x16x32: A = 16 rows x 32 bins from LDS, B = D split
//      into bfloat16 hi/lo halves packed as 16 columns [D_hi | D_lo], so one
//      instruction gives both products and N_V = C[:, j] + C[:, 8 + j];
//   3. the per-wave N_V partials are summed in LDS (fixed order) and the row
//      rule updates V in float64 registers: Lee-Seung MU, HALS, or (ANLS) the
//      exact NNLS of each row, 32 lanes per row enumerating the supports;
//      (N_D alone: steps 2 and 3 are skipped and the given V is used);
//   4. N_D += P^T V_new on MFMA 16x16x16: A = P^T (16 bins x 16 rows, read
//      transposed from the LDS tile), B = [V_hi | V_lo]; the accumulators
//      stay in registers for the whole pass;
//   5. on objective iterations, V_new D^T is rebuilt on MFMA 16x16x32 from
//      [V_hi | V_lo | V_hi] x [D_hi ; D_hi ; D_lo] and ||P - V_new D^T||^2 is
//      accumulated against the same bfloat16 P values (MU, HALS); an ANLS
//      pass solves each row exactly for D' = D_hi + D_lo (inverses of G_D'),
//      so a row's objective is ||p_row||^2 + 2 q_min with q_min the least
//      cost of its enumeration, and ||p_row||^2 comes from the N_V operands.
// p is read from HBM exactly once per iteration; everything else stays on chip.
#include "nmf_common.hpp"

namespace hsn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBThreads = 512;
constexpr int kBWaves = kBThreads / 64;
constexpr int kBRows = 16;
constexpr int kMaxLdb = 2048;
// Every wave owns exactly NW k-steps of 32 bins (NW = 1, 2, 4 or 8), so the
// row of the LDS tile and the operand images are padded to 256 NW bins; bins
// at or beyond ldb load as zeros.  The load code is branch-free (clamped
// address + select) so the compiler can count outstanding loads exactly and
// the prefetched tiles stay in flight across the tile's compute.  With NW <= 4
// the registers left over hold a second tile of loads in flight (NBUF = 2);
// with NW = 8 a second tile did not fit (MU, HALS) or ran slower (ANLS:
// 8.1 against 7.7 ms at 2000 bins).
__host__ __device__ inline int64_t bf16_ldb_pad(int64_t ldb) {
  const int64_t nw = (ldb + 255) / 256;
  return 256 * (nw <= 1 ? 1 : nw <= 2 ? 2 : nw <= 4 ? 4 : 8);
}

// Row pitch of the LDS tile in bytes: 4 (mod 64) banks past a whole row, so
// the 16-byte reads of the N_V operand (16 rows, one 16-byte chunk each per
// 16 lanes) and the 2-byte transposed reads of the N_D operand (rows 4 g + q,
// 16 bins, g = lane / 16) fall on distinct banks.
__host__ __device__ inline int bf16_pitch(int64_t ldb) { return int(2 * bf16_ldb_pad(ldb) + 16); }

struct Bf16Lds {
  int tile, db1, red, vsp, vnw, vold, gd, obj, hsum, ginv, total;
};

// The inverses of G_D's principal submatrices (fused ANLS) are staged in LDS
// for K <= 6 (tri(K) x 2^K doubles, at most 10.5 KB) and read from the caches above.
__host__ __device__ constexpr bool bf16_inv_in_lds(int K) { return K <= 6; }

__host__ __device__ inline Bf16Lds bf16_lds_layout(int64_t ldb, int K, bool anls = false) {
  Bf16Lds L;
  int o = 0;
  L.tile = o;
  o += kBRows * bf16_pitch(ldb);
  o = (o + 15) & ~15;
  L.db1 = o;
  o += int(bf16_ldb_pad(ldb) / 32) * 64 * 16;
  L.red = o;
  o += kBWaves * 16 * 16 * 4;
  L.vsp = o;
  o += 16 * 16 * 2;
  L.vnw = o;
  o += 16 * 8 * 4;
  L.vold = o;
  o += 16 * 8 * 4;
  L.gd = o;
  o += 64 * 8;
  L.obj = o;
  o += kBWaves * 8;
  L.hsum = o;
  o += anls ? kBRows * 8 * 4 : 0;
  o = (o + 15) & ~15;
  L.ginv = o;
  o += (anls && bf16_inv_in_lds(K)) ? (1 << K) * tri(K) * 8 : 0;
  L.total = o;
  return L;
}

// The pass of one decomposition by workgroup blk of nblk (persistent,
// tiles blk, blk + nblk, ...); smem: the dynamic LDS (bf16_lds_layout).
template <int K, int MODE, bool OBJ, int NW, int NBUF>
__device__ __forceinline__ void pass_bf16_body(const uint16_t *__restrict__ Pb, int64_t ldb, int64_t n_p, int n_k,
                                               float *__restrict__ V, const uint4 *__restrict__ db1g,
                                               const uint4 *__restrict__ db3g, const double *__restrict__ GD,
                                               const double *__restrict__ chol, float *__restrict__ part_nd,
                                               double *__restrict__ part_gv, double *__restrict__ part_obj,
                                               NmfCtrl *__restrict__ ctrl, int iter,
                                               const double *__restrict__ ginv, int blk, int nblk,
                                               char *__restrict__ smem) {
  if (iter >= ctrl->stop_at) return;
  const Bf16Lds L = bf16_lds_layout(ldb, K, MODE == kModeANLS);
  char *tileL = smem + L.tile;
  uint4 *db1L = reinterpret_cast<uint4 *>(smem + L.db1);
  float *red = reinterpret_cast<float *>(smem + L.red);        // [8][16][16], [wave][col][row]
  uint16_t *vsp = reinterpret_cast<uint16_t *>(smem + L.vsp);  // [16][16]  [V_hi | V_lo]
  float *vnw = reinterpret_cast<float *>(smem + L.vnw);        // [16][8]
  float *vold = reinterpret_cast<float *>(smem + L.vold);      // [16][K] V of the tile before the update
  double *gd_s = reinterpret_cast<double *>(smem + L.gd);
  double *obj_s = reinterpret_cast<double *>(smem + L.obj);

  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  constexpr int kKSW = NW;
  constexpr int nw = NW;
  const int pitch = bf16_pitch(ldb);
  const int nks = kBWaves * NW;  // k-steps of the padded row
  const int s0 = w * NW;
  constexpr int cpr = 4 * NW;   // 16-byte chunks per row in this wave's bins

  if constexpr (MODE != kModeND)  // N_D alone needs no operand image of D
    for (int i = t; i < nks * 64; i += kBThreads) db1L[i] = db1g[i];
  for (int i = t; i < 16 * 16; i += kBThreads) vsp[i] = 0;
  if (t < K * K) gd_s[t] = GD[t];
  float *hsum = reinterpret_cast<float *>(smem + L.hsum);  // [16][8]
  const double *ginv_s = ginv;
  if constexpr (MODE == kModeANLS && bf16_inv_in_lds(K)) {
    // entry-major, stride 2^K
    double *g = reinterpret_cast<double *>(smem + L.ginv);
    for (int i = t; i < (1 << K) * tri(K); i += kBThreads) g[i] = ginv[(i >> K) * kInvStride + (i & ((1 << K) - 1))];
    ginv_s = g;
  }

  f32x4 acc2[2 * kKSW];
#pragma unroll
  for (int b = 0; b < 2 * kKSW; ++b) acc2[b] = f32x4{0.f, 0.f, 0.f, 0.f};
  double gv = 0.0, obj = 0.0;

  uint4 prA[kKSW], prB[kKSW];
  float vA = 0.0f, vB = 0.0f;  // the tile's V values (thread t < 16 K holds one)
  // Tile loads go through buffer descriptors covering the tile's valid rows:
  // rows past n_p and bins past ldb (offset pushed out of range) read as 0
  // without a branch, so the loads stay unconditional and in flight.
  auto load_tile = [&](uint4 (&pr)[kKSW], float &vv, int64_t row0) {
    const int64_t rows = (n_p - row0) < kBRows ? (n_p - row0) : kBRows;
    if constexpr (MODE != kModeANLS) {  // an exact row solve does not read the old V
      const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(V) + row0 * K, 0, int(rows * K * 4), 0x00020000);
      vv = __builtin_bit_cast(float,
                              __builtin_amdgcn_raw_buffer_load_b32(rv, t < kBRows * K ? 4 * t : 0x7FFFFFF0, 0, 0));
    }
    const __amdgpu_buffer_rsrc_t rp = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t *>(Pb) + row0 * ldb, 0, int(rows * ldb * 2), 0x00020000);
#pragma unroll
    for (int i = 0; i < kKSW; ++i) {
      const int c = lane + 64 * i;
      const int r = c / cpr, cc = c % cpr;
      const int col = 32 * s0 + 8 * cc;
      const int off = (col < ldb) ? int(r * ldb + col) * 2 : 0x7FFFFFF0;
      pr[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rp, off, 0, 0));
    }
  };

  // NBUF register buffers keep NBUF tiles of loads in flight per wave.
  const int64_t n_tiles = (n_p + kBRows - 1) / kBRows;
  const int64_t G = nblk;
  if (int64_t(blk) < n_tiles) load_tile(prA, vA, int64_t(blk) * kBRows);
  if (NBUF == 2 && int64_t(blk) + G < n_tiles) load_tile(prB, vB, (int64_t(blk) + G) * kBRows);
  __syncthreads();

  auto do_tile = [&](uint4 (&pr)[kKSW], float &vv, int64_t tile) {
    const int64_t row0 = tile * kBRows;
    // 1. this wave's bins of the tile -> LDS (16-byte stores)
#pragma unroll
    for (int i = 0; i < kKSW; ++i) {
      if (i < nw) {
        const int c = lane + 64 * i;
        const int r = c / cpr, cc = c - (c / cpr) * cpr;
        *reinterpret_cast<uint4 *>(tileL + r * pitch + 2 * (32 * s0 + 8 * cc)) = pr[i];
      }
    }
    if (MODE != kModeANLS && t < kBRows * K) vold[t] = vv;
    // prefetch the tile NBUF steps ahead into the same registers
    if (tile + NBUF * G < n_tiles) load_tile(pr, vv, (tile + NBUF * G) * kBRows);
    // A wave reads only its own bins of the tile, so only vold (not used by
    // the exact solves) needs the barrier.
    if constexpr (MODE != kModeANLS) __syncthreads();

    // 2. N_V partial over this wave's bins (not for N_D alone)
    if constexpr (MODE != kModeND) {
    f32x4 acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < kKSW; ++i) {
      if (i < nw) {
        const int s = s0 + i;
        const uint4 av =
            *reinterpret_cast<const uint4 *>(tileL + (lane & 15) * pitch + 2 * (32 * s + 8 * (lane >> 4)));
        const uint4 bv = db1L[s * 64 + lane];
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                       acc1, 0, 0, 0);
        if constexpr (OBJ && MODE == kModeANLS) {
          // ||p||^2 of the tile: every element once over (wave, k-step, lane);
          // the squares are exact in float32
          const uint32_t wd[4] = {av.x, av.y, av.z, av.w};
          float sq = 0.0f;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float v = bf16_bits_to_f32(uint16_t(wd[e >> 1] >> (16 * (e & 1))));
            sq = fmaf(v, v, sq);
          }
          obj += double(sq);
        }
      }
    }
    // column-major per wave (red[w][col][row]): the lane's four rows are one 16-byte store
    *reinterpret_cast<f32x4 *>(red + (w * 16 + (lane & 15)) * 16 + 4 * (lane >> 4)) = acc1;
    __syncthreads();
    }

    // 3. row rule
    if (MODE == kModeND) {
      // N_D = P^T V for the given V: the tile's V as loaded
      if (t < kBRows * K) {
        const int r = t / K, j = t - (t / K) * K;
        const float vn = (row0 + r < n_p) ? vold[t] : 0.0f;
        vnw[r * 8 + j] = vn;
        vsp[r * 16 + j] = bf_hi(vn);
        vsp[r * 16 + 8 + j] = bf_lo(vn);
      }
    } else if (MODE == kModeANLS) {
      // exact NNLS of the 16 rows: h into LDS, then 32 lanes per row
      if (t < kBRows * K) {
        const int r = t / K, j = t - (t / K) * K;
        float s = 0.0f;
#pragma unroll
        for (int ww = 0; ww < kBWaves; ++ww) s += red[(ww * 16 + j) * 16 + r] + red[(ww * 16 + 8 + j) * 16 + r];
        hsum[r * 8 + j] = s;
      }
      __syncthreads();
      const int r = t >> 5, l = t & 31;
      const int64_t row = row0 + r;
      float h[K];
#pragma unroll
      for (int j = 0; j < K; ++j) h[j] = hsum[r * 8 + j];
      double qmin = 0.0;
      const double xl =
          nnls_enum_group<K, bf16_inv_in_lds(K) ? (1 << K) : kInvStride>(ginv_s, h, l, OBJ ? &qmin : nullptr);
      // the row's objective at its exact solution is ||p_row||^2 + 2 qmin
      if (OBJ && l == 0 && row < n_p) obj += 2.0 * qmin;
      if (l < K) {
        float vn = float(xl);
        if (row >= n_p) vn = 0.0f;
        if (row < n_p) V[row * K + l] = vn;
        vnw[r * 8 + l] = vn;
        vsp[r * 16 + l] = bf_hi(vn);
        vsp[r * 16 + 8 + l] = bf_lo(vn);
      }
    } else if (MODE == kModeHALS) {
      if (t < kBRows) {
        const int r = t;
        const int64_t row = row0 + r;
        double h[K], x[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
          float s = 0.0f;
#pragma unroll
          for (int ww = 0; ww < kBWaves; ++ww) s += red[(ww * 16 + j) * 16 + r] + red[(ww * 16 + 8 + j) * 16 + r];
          h[j] = s;
          x[j] = (row < n_p) ? double(vold[r * K + j]) : 0.0;
        }
        hals_row<K>(gd_s, h, x);
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const float vn = (row < n_p) ? float(x[j]) : 0.0f;
          if (row < n_p) V[row * K + j] = vn;
          vnw[r * 8 + j] = vn;
          vsp[r * 16 + j] = bf_hi(vn);
          vsp[r * 16 + 8 + j] = bf_lo(vn);
        }
      }
    } else if (t < kBRows * K) {
      const int r = t / K, j = t - (t / K) * K;
      const int64_t row = row0 + r;
      float s = 0.0f;
#pragma unroll
      for (int ww = 0; ww < kBWaves; ++ww) s += red[(ww * 16 + j) * 16 + r] + red[(ww * 16 + 8 + j) * 16 + r];
      float vn = 0.0f;
      if (row < n_p) {
        float vr[K];
#pragma unroll
        for (int i = 0; i < K; ++i) vr[i] = vold[r * K + i];
        double den = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) den += double(vr[i]) * gd_s[i * K + j];
        vn = float(double(vr[j]) * double(s) / fmax(den, 1e-300));
        V[row * K + j] = vn;
      }
      vnw[r * 8 + j] = vn;
      vsp[r * 16 + j] = bf_hi(vn);
      vsp[r * 16 + 8 + j] = bf_lo(vn);
    }
    __syncthreads();

    // 4. N_D += P^T V_new (and 5. the residual on objective iterations)
    if (t < K * K) {
      const int i = t / K, j = t - (t / K) * K;
      float s = 0.0f;
#pragma unroll
      for (int r = 0; r < kBRows; ++r) s = fmaf(vnw[r * 8 + i], vnw[r * 8 + j], s);
      gv += double(s);
    }
    // [V_hi | V_lo] operand, lane (g, n): rows 4 g .. 4 g + 3 of column n, by
    // one transposed 8-byte read (lane addressing as for P^T below)
    const s16x4 b2 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
        (__attribute__((address_space(3))) s16x4 *)(vsp + (4 * (lane >> 4) + ((lane >> 2) & 3)) * 16 + 4 * (lane & 3)));
    bf16x8 a3;
    // the reconstruction objective (MU, HALS); an ANLS pass has its objective
    // from the row solves
    constexpr bool RECON = OBJ && MODE != kModeANLS;
    if (RECON) {
      const int g = lane >> 4, row = lane & 15;
      uint16_t u[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) u[e] = (g == 3) ? 0 : vsp[row * 16 + (g == 1 ? 8 : 0) + e];
      a3 = __builtin_bit_cast(bf16x8, make_uint4(u[0] | (uint32_t(u[1]) << 16), u[2] | (uint32_t(u[3]) << 16),
                                                 u[4] | (uint32_t(u[5]) << 16), u[6] | (uint32_t(u[7]) << 16)));
    }
    float objf = 0.0f;
#pragma unroll
    for (int i = 0; i < kKSW; ++i) {
      if (i < nw) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int bin0 = 32 * (s0 + i) + 16 * hh;
          // P^T operand, lane (g, n) = (lane >> 4, lane & 15): rows 4 g .. 4 g + 3
          // of bin bin0 + n, by one transposed 8-byte read: lane
          // (g, j, m) = (lane >> 4, (lane >> 2) & 3, lane & 3) addresses bins
          // bin0 + 4 m .. + 3 of row 4 g + j, and within each 16 lanes the read
          // hands lane n element j of lane 4 j + n / 4, item n % 4.
          const s16x4 a2 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
              (__attribute__((address_space(3))) s16x4 *)(tileL + (4 * (lane >> 4) + ((lane >> 2) & 3)) * pitch +
                                                          2 * (bin0 + 4 * (lane & 3))));
          acc2[2 * i + hh] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, b2, acc2[2 * i + hh], 0, 0, 0);
          if (RECON) {
            const uint4 b3 = db3g[(bin0 / 16) * 64 + lane];
            f32x4 rec = {0.f, 0.f, 0.f, 0.f};
            rec = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, __builtin_bit_cast(bf16x8, b3), rec, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float df = bf16_bits_to_f32(uint16_t(a2[q])) - rec[q];
              objf = fmaf(df, df, objf);
            }
          }
        }
      }
    }
    if (RECON) obj += double(objf);
  };
  if (NBUF == 2) {
    for (int64_t tile = blk; tile < n_tiles; tile += 2 * G) {
      do_tile(prA, vA, tile);
      if (tile + G < n_tiles) do_tile(prB, vB, tile + G);
    }
  } else {
    for (int64_t tile = blk; tile < n_tiles; tile += G) do_tile(prA, vA, tile);
  }

  // Partials: N_D[bin][j] = C[bin][j] + C[bin][8 + j] (lanes n and n + 8).
  float *dst = part_nd + size_t(blk) * n_k * K;
  const int n = lane & 15;
#pragma unroll
  for (int i = 0; i < kKSW; ++i) {
    if (i < nw) {
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float v = acc2[2 * i + hh][q];
          const float other = __shfl_xor(v, 8, 64);
          const int bin = 32 * (s0 + i) + 16 * hh + 4 * (lane >> 4) + q;
          if (n < K && bin < n_k) dst[size_t(bin) * K + n] = v + other;
        }
      }
    }
  }
  if (t < K * K) part_gv[size_t(blk) * K * K + t] = gv;
  if (OBJ) {
    obj = wave_sum_all(obj);
    if (lane == 0) obj_s[w] = obj;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int ww = 0; ww < kBWaves; ++ww) s += obj_s[ww];
      part_obj[blk] = s;
    }
  }
}


template <int K, int MODE, bool OBJ, int NW, int NBUF>
__global__ __launch_bounds__(kBThreads) void pass_bf16_kernel(const uint16_t *__restrict__ Pb, int64_t ldb,
                                                              int64_t n_p, int n_k, float *__restrict__ V,
                                                              const uint4 *__restrict__ db1g,
                                                              const uint4 *__restrict__ db3g,
                                                              const double *__restrict__ GD,
                                                              const double *__restrict__ chol,
                                                              float *__restrict__ part_nd,
                                                              double *__restrict__ part_gv,
                                                              double *__restrict__ part_obj,
                                                              NmfCtrl *__restrict__ ctrl, int iter,
                                                              const double *__restrict__ ginv) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  pass_bf16_body<K, MODE, OBJ, NW, NBUF>(Pb, ldb, n_p, n_k, V, db1g, db3g, GD, chol, part_nd, part_gv, part_obj, ctrl,
                                         iter, ginv, int(blockIdx.x), int(gridDim.x), smem);
}

// Batched MU iterations on the bfloat16 p: one launch over the instances
// d[0 .. n_inst) of one (K, k-step class) group; block b belongs to the
// instance whose range [wg0b, wg0b + n_wgb) holds it (wg0b counted from the
// group's first instance) and runs that instance's pass as workgroup
// b - wg0b of n_wgb, so each instance computes what its own call computes.
template <int K, bool OBJ, int NW, int NBUF>
__global__ __launch_bounds__(kBThreads) void batched_pass_bf16_kernel(const BatchInst *__restrict__ d, int n_inst,
                                                                      int iter_local) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int i = batch_find(n_inst, int(blockIdx.x), [&](int j) { return d[j].wg0b; });
  const BatchInst &b = d[i];
  const int wg = int(blockIdx.x) - b.wg0b;
  if (wg >= b.n_wgb) return;
  const int iter = b.ctrl->iter_base + iter_local;
  const uint4 *db1 = reinterpret_cast<const uint4 *>(b.img);
  const uint4 *db3 = db1 + (bf16_ldb_pad(b.ldb) / 32) * 64;
  pass_bf16_body<K, kModeMU, OBJ, NW, NBUF>(b.Pb, b.ldb, b.n_p, b.n_k, b.V, db1, db3, b.gd, b.chol, b.part_nd,
                                            b.part_gv, b.part_obj, b.ctrl, iter, nullptr, wg, b.n_wgb, smem);
}

template <int K, int MODE, bool OBJ, int NW, int NBUF>
static bool launch_bf16_inst(int n_wg, hipStream_t st, const uint16_t *Pb, int64_t ldb, int64_t n_p, int n_k,
                             float *V, const uint4 *db1, const uint4 *db3, const double *GD, const double *chol,
                             float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                             const double *ginv) {
  const int lds = bf16_lds_layout(ldb, K, MODE == kModeANLS).total;
  static bool attr_set = false;
  if (!attr_set) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&pass_bf16_kernel<K, MODE, OBJ, NW, NBUF>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
      return false;
    attr_set = true;
  }
  pass_bf16_kernel<K, MODE, OBJ, NW, NBUF><<<n_wg, kBThreads, lds, st>>>(Pb, ldb, n_p, n_k, V, db1, db3, GD, chol, part_nd,
                                                                part_gv, part_obj, ctrl, iter, ginv);
  return true;
}

// NB_MU: tiles in flight for MU and HALS (their objective reconstruction
// needs registers), NB_X: for ANLS and N_D alone.
template <int K, int NW, int NB_MU, int NB_X>
static bool launch_bf16_kw(int mode, bool obj, int n_wg, hipStream_t st, const uint16_t *Pb, int64_t ldb, int64_t n_p,
                           int n_k, float *V, const uint4 *db1, const uint4 *db3, const double *GD, const double *chol,
                           float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                           const double *ginv) {
#define HSN_INST(M_, O_, NB_) \
  launch_bf16_inst<K, M_, O_, NW, NB_>(n_wg, st, Pb, ldb, n_p, n_k, V, db1, db3, GD, chol, part_nd, part_gv, part_obj, \
                                       ctrl, iter, ginv)
  if (mode == kModeANLS) return obj ? HSN_INST(kModeANLS, true, NB_X) : HSN_INST(kModeANLS, false, NB_X);
  if (mode == kModeND) return HSN_INST(kModeND, false, NB_X);
  if (mode == kModeMU) return obj ? HSN_INST(kModeMU, true, NB_MU) : HSN_INST(kModeMU, false, NB_MU);
  if (mode == kModeHALS) return obj ? HSN_INST(kModeHALS, true, NB_MU) : HSN_INST(kModeHALS, false, NB_MU);
  return false;
#undef HSN_INST
}

template <int K>
static bool launch_bf16_k(int mode, bool obj, int n_wg, hipStream_t st, const uint16_t *Pb, int64_t ldb, int64_t n_p,
                          int n_k, float *V, const uint4 *db1, const uint4 *db3, const double *GD, const double *chol,
                          float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                          const double *ginv) {
  const int64_t nw = bf16_ldb_pad(ldb) / 256;
#define HSN_NW(NW_, NB_MU_, NB_X_)                                                                                 \
  if (nw == NW_)                                                                                                   \
    return launch_bf16_kw<K, NW_, NB_MU_, NB_X_>(mode, obj, n_wg, st, Pb, ldb, n_p, n_k, V, db1, db3, GD, chol,    \
                                                 part_nd, part_gv, part_obj, ctrl, iter, ginv);
  HSN_NW(1, 2, 2) HSN_NW(2, 2, 2) HSN_NW(4, 2, 2) HSN_NW(8, 1, 1)
#undef HSN_NW
  return false;
}

// Row pitch of the operand images of D (padded to the wave split) and their
// size in uint16 (see nmf_iter.hip).
int64_t bf16_image_ldb(int64_t ldb) { return bf16_ldb_pad(ldb); }
size_t bf16_image_elems(int64_t ldb) {
  const int64_t l = bf16_ldb_pad(ldb);
  return size_t(l / 32) * 64 * 8 + size_t(l / 16) * 64 * 8;
}

bool launch_pass_bf16(int K, int mode, bool obj, int n_wg, hipStream_t st, const uint16_t *Pb, int64_t ldb,
                      int64_t n_p, int n_k, float *V, const double *GD, const double *chol, const uint16_t *img,
                      float *part_nd, double *part_gv, double *part_obj, NmfCtrl *ctrl, int iter,
                      const double *ginv) {
  if (ldb > kMaxLdb || ldb % 32 != 0 || K < 1 || K > 8 ||
      (mode != kModeMU && mode != kModeHALS && mode != kModeANLS && mode != kModeND) || (mode == kModeANLS && !ginv))
    return false;
  const uint4 *db1 = reinterpret_cast<const uint4 *>(img);
  const uint4 *db3 = db1 + (bf16_ldb_pad(ldb) / 32) * 64;
  switch (K) {
#define HSN_K(KK)                                                                                                  \
  case KK:                                                                                                         \
    return launch_bf16_k<KK>(mode, obj, n_wg, st, Pb, ldb, n_p, n_k, V, db1, db3, GD, chol, part_nd, part_gv,     \
                             part_obj, ctrl, iter, ginv);
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
  return false;
}

template <int K, int NW, int NBUF>
static bool launch_batched_bf16_inst(bool obj, int n_blocks, int lds, hipStream_t st, const BatchInst *d,
                                     int n_inst, int iter_local) {
  static bool attr_set[2] = {false, false};
  const void *fn = obj ? reinterpret_cast<const void *>(&batched_pass_bf16_kernel<K, true, NW, NBUF>)
                       : reinterpret_cast<const void *>(&batched_pass_bf16_kernel<K, false, NW, NBUF>);
  if (!attr_set[obj]) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) return false;
    attr_set[obj] = true;
  }
  if (obj)
    batched_pass_bf16_kernel<K, true, NW, NBUF><<<n_blocks, kBThreads, lds, st>>>(d, n_inst, iter_local);
  else
    batched_pass_bf16_kernel<K, false, NW, NBUF><<<n_blocks, kBThreads, lds, st>>>(d, n_inst, iter_local);
  return true;
}

// One batched MU pass over a (K, k-step class) group: nw = bf16_ldb_pad(ldb)
// / 256 of its instances (tiles in flight as for the single-instance MU pass).
bool launch_batched_pass_bf16(int K, int nw, bool obj, int n_blocks, hipStream_t st, const BatchInst *d, int n_inst,
                              int iter_local) {
  if (K < 1 || K > 8) return false;
  const int lds = bf16_lds_layout(256 * int64_t(nw), K, false).total;
  switch (K) {
#define HSN_K(KK)                                                                                              \
  case KK:                                                                                                     \
    if (nw == 1) return launch_batched_bf16_inst<KK, 1, 2>(obj, n_blocks, lds, st, d, n_inst, iter_local);    \
    if (nw == 2) return launch_batched_bf16_inst<KK, 2, 2>(obj, n_blocks, lds, st, d, n_inst, iter_local);    \
    if (nw == 4) return launch_batched_bf16_inst<KK, 4, 2>(obj, n_blocks, lds, st, d, n_inst, iter_local);    \
    if (nw == 8) return launch_batched_bf16_inst<KK, 8, 1>(obj, n_blocks, lds, st, d, n_inst, iter_local);    \
    return false;
    HSN_K(1) HSN_K(2) HSN_K(3) HSN_K(4) HSN_K(5) HSN_K(6) HSN_K(7) HSN_K(8)
#undef HSN_K
  }
  return false;
}

int bf16_k_steps_class(int64_t ldb) { return int(bf16_ldb_pad(ldb) / 256); }

int pass_bf16_wgs(hsn_ctx *ctx, int64_t n_p) {
  const int64_t n_tiles = (n_p + kBRows - 1) / kBRows;
  return int(std::min<int64_t>(n_tiles, ctx->num_cu));
}

}  // namespace hsn
