// Subspace expansion, eq. (6): x^h = x^s (D^s)^T over a voxel range and a
// bin range.  Output-write bound: each thread owns one bin b (coalesced
// stores along b), keeps D[b][:] in registers and walks a run of voxels
// whose K coefficients are uniform across the block.
#include "common.hpp"

namespace {

constexpr int kBins = 256;   // threads per block, one bin each
constexpr int kVox = 32;     // voxels per block

template <int K>
__global__ __launch_bounds__(kBins) void rehydrate_kernel(const float *__restrict__ xs, const float *__restrict__ D,
                                                          int64_t vb, int64_t ve, int64_t bb, int64_t be,
                                                          float *__restrict__ xh, int64_t ldh) {
  const int64_t b = bb + int64_t(blockIdx.x) * kBins + threadIdx.x;
  const int64_t v0 = vb + int64_t(blockIdx.y) * kVox;
  if (b >= be) return;
  float d[K];
#pragma unroll
  for (int q = 0; q < K; ++q) d[q] = D[b * K + q];
  const int64_t v1 = v0 + kVox < ve ? v0 + kVox : ve;
  for (int64_t v = v0; v < v1; ++v) {
    float acc = 0.0f;
#pragma unroll
    for (int q = 0; q < K; ++q) acc = fmaf(xs[v * K + q], d[q], acc);
    xh[(v - vb) * ldh + (b - bb)] = acc;
  }
}

template <int K>
void launch(const float *xs, const float *D, int64_t vb, int64_t ve, int64_t bb, int64_t be, float *xh, int64_t ldh,
            hipStream_t st) {
  dim3 grid(unsigned((be - bb + kBins - 1) / kBins), unsigned((ve - vb + kVox - 1) / kVox));
  rehydrate_kernel<K><<<grid, kBins, 0, st>>>(xs, D, vb, ve, bb, be, xh, ldh);
}

}  // namespace

extern "C" hsn_status hsn_rehydrate(hsn_ctx *ctx, const float *xs, const float *D, int64_t n_x, int64_t n_k, int k,
                                    int64_t vox_begin, int64_t vox_end, int64_t bin_begin, int64_t bin_end, float *xh,
                                    int64_t ldh, void *stream) {
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (!xs || !D || !xh) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "rehydrate: xs, D and xh are required");
  if (k < 1 || k > 8) return hsn::fail(ctx, HSN_ERR_SHAPE, "rehydrate: k must be in 1..8");
  if (vox_begin < 0 || vox_end > n_x || vox_begin >= vox_end || bin_begin < 0 || bin_end > n_k ||
      bin_begin >= bin_end)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "rehydrate: empty or out-of-range voxel/bin range");
  if (ldh < bin_end - bin_begin) return hsn::fail(ctx, HSN_ERR_INVALID_ARG, "rehydrate: ldh too small");
  if ((vox_end - vox_begin + kVox - 1) / kVox > 65535LL * 1024)
    return hsn::fail(ctx, HSN_ERR_SHAPE, "rehydrate: voxel range too large for one call");
  hsn::DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nvb = (vox_end - vox_begin + kVox - 1) / kVox;
  // grid.y is limited to 65535: split long voxel ranges into slabs.
  for (int64_t s0 = 0; s0 < nvb; s0 += 65535) {
    const int64_t vb = vox_begin + s0 * kVox;
    const int64_t ve = std::min<int64_t>(vox_end, vb + 65535LL * kVox);
    float *out = xh + (vb - vox_begin) * ldh;
    switch (k) {
      case 1: launch<1>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
      case 2: launch<2>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
      case 3: launch<3>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
      case 4: launch<4>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
      case 5: launch<5>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
      case 6: launch<6>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
      case 7: launch<7>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
      default: launch<8>(xs, D, vb, ve, bin_begin, bin_end, out, ldh, st); break;
    }
    HSN_LAUNCHED(ctx);
  }
  return HSN_OK;
}
