// Learned warm start for the sigma_min run: a 4-layer 3x3 CNN
// (2 -> 64 -> 64 -> 64 -> 6 channels, ReLU after the first three) that maps
// the two coefficient fields of a hydro-mechanical grid to a start vector.
// It changes nothing in the estimator's arithmetic; a poor start only costs
// iterations, and the caller keeps a random start beside it.
//
// gfx950 implementation: activations and weights in bfloat16, NHWC with the
// channel count padded to a multiple of 8; every convolution (forward and
// input gradient) is an implicit GEMM on v_mfma_f32_16x16x32_bf16 with
// float32 accumulation; the weight gradient is an MFMA GEMM over pixels cut
// into slices whose partials are added in slice order (deterministic). Adam
// updates float32 master weights, which are then repacked into the bfloat16
// layouts of the forward and input-gradient convolutions.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "condest.h"
#include "internal.hpp"

using namespace condest;

#define NCHK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(COND_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kLayers = 4;
constexpr int kCh[kLayers + 1] = {2, 64, 64, 64, 6};
constexpr int kPad[kLayers + 1] = {8, 64, 64, 64, 16};  // padded channel counts
constexpr int kSlicePix = 256;                          // pixels per weight-gradient slice

__host__ __device__ constexpr int kpad(int cin_pad) { return (9 * cin_pad + 31) / 32 * 32; }

// float -> bfloat16, round to nearest even
__device__ __forceinline__ u16 to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return static_cast<u16>((u >> 16) | 0x40);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<u16>(u >> 16);
}
__device__ __forceinline__ float from_bf16(u16 h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }

union Frag {
  bf16x8 v;
  uint4 q;
  u16 h[8];
};

// ------------------------------------------------------------------ prep
// cell fields (log10 eta, log10 k), float64 [B][2][S-1][S-1] -> node input
// [B][S][S][8] bfloat16: mean of the adjacent cells (edge replicated), then
// centred and scaled; channels 2..7 are zero.
__global__ void prep_k(const double* __restrict__ cells, u16* __restrict__ act0, int B, int S) {
  const long long n = static_cast<long long>(B) * S * S;
  const long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const int b = static_cast<int>(i / (S * S));
  const int r = static_cast<int>(i % (S * S));
  const int y = r / S, x = r % S;
  const int C = S - 1;
  const double centre[2] = {21.0, -16.0}, half[2] = {3.0, 4.0};
  u16 out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int f = 0; f < 2; ++f) {
    const double* c = cells + (static_cast<long long>(b) * 2 + f) * C * C;
    double s = 0.0;
    for (int dx = -1; dx <= 0; ++dx)
      for (int dy = -1; dy <= 0; ++dy) {
        int cy = y + dy, cx = x + dx;
        cy = cy < 0 ? 0 : (cy > C - 1 ? C - 1 : cy);
        cx = cx < 0 ? 0 : (cx > C - 1 ? C - 1 : cx);
        s += c[cy * C + cx];
      }
    out[f] = to_bf16(static_cast<float>((0.25 * s - centre[f]) / half[f]));
  }
  uint4 q;
  std::memcpy(&q, out, 16);
  reinterpret_cast<uint4*>(act0)[i] = q;
}

// ------------------------------------------------------------------ conv
// out[p, co] = sum_{tap, ci} in[p + tap offset, ci] * wt[co][tap * CIN + ci]
// A block of 4 waves takes 64 pixels; the packed weights ([COUT][KP]
// bfloat16) are first staged in LDS, then each wave computes 16 pixels x all
// COUT channels: per step of 32 k-values it loads one A fragment (its 16
// pixels' inputs) and reuses it for COUT/16 MFMAs whose B fragments come from
// LDS. MFMA v_mfma_f32_16x16x32_bf16 lane layout: A lane l holds row l % 16,
// k = 8 (l / 16) .. + 7; B lane l holds column l % 16, same k; the result
// lane l holds column l % 16, rows 4 (l / 16) .. + 3.
// EPI 0: + bias, ReLU, bfloat16 out; 1: + bias, float32 out (last layer);
// 2: times (mask > 0), bfloat16 out (input gradient through a ReLU).
constexpr int kConvWaves = 8;

template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(64 * kConvWaves) void conv_k(const u16* __restrict__ in,
                                                          const u16* __restrict__ wt,
                                                          const float* __restrict__ bias,
                                                          const u16* __restrict__ mask,
                                                          void* __restrict__ out, int B, int S) {
  constexpr int K = 9 * CIN, KP = kpad(CIN), NB = COUT / 16;
  __shared__ uint4 w_sh[COUT * KP / 8];
  for (int i = threadIdx.x; i < COUT * KP / 8; i += 64 * kConvWaves)
    w_sh[i] = reinterpret_cast<const uint4*>(wt)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long npix = static_cast<long long>(B) * S * S;
  const long long p0 = (static_cast<long long>(blockIdx.x) * kConvWaves + wave) * 16;
  if (p0 >= npix) return;  // no barrier follows
  const long long pa = p0 + (lane & 15);
  const bool pin = pa < npix;
  const int b = pin ? static_cast<int>(pa / (S * S)) : 0;
  const int rr = pin ? static_cast<int>(pa % (S * S)) : 0;
  const int y = rr / S, x = rr % S;
  const int kq = 8 * (lane >> 4);
  f32x4 acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int ks = 0; ks < KP; ks += 32) {
    const int k0 = ks + kq;
    Frag a;
    a.q = make_uint4(0, 0, 0, 0);
    if (pin && k0 < K) {
      const int tap = k0 / CIN, ci0 = k0 % CIN;
      const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
      if (yy >= 0 && yy < S && xx >= 0 && xx < S)
        a.q = *reinterpret_cast<const uint4*>(in + ((static_cast<long long>(b) * S + yy) * S + xx) * CIN + ci0);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      Frag w;
      w.q = w_sh[((j * 16 + (lane & 15)) * KP + k0) / 8];
      acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, w.v, acc[j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int co = jb * 16 + (lane & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long long p = p0 + 4 * (lane >> 4) + j;
      if (p >= npix) continue;
      float v = acc[jb][j];
      if (EPI == 0) {
        v += bias[co];
        v = v > 0.f ? v : 0.f;
        static_cast<u16*>(out)[p * COUT + co] = to_bf16(v);
      } else if (EPI == 1) {
        v += bias[co];
        static_cast<float*>(out)[p * COUT + co] = v;
      } else {
        v = from_bf16(mask[p * COUT + co]) > 0.f ? v : 0.f;
        static_cast<u16*>(out)[p * COUT + co] = to_bf16(v);
      }
    }
  }
}

// ---------------------------------------------------------- weight gradient
// part[slice][r][co] = sum over the slice's pixels p of in[p + tap(r), ci(r)] * g[p, co]
// for r = tap * CIN + ci < 9 CIN, and of g[p, co] alone for r = 9 CIN (the
// bias row); MFMA with M = 16 rows r, N = 16 channels, K = 32 pixels a step.
__host__ __device__ constexpr int wrows(int cin) { return (9 * cin + 1 + 15) / 16 * 16; }

template <int CIN, int COUT>
__global__ __launch_bounds__(64) void wgrad_k(const u16* __restrict__ in, const u16* __restrict__ g,
                                              float* __restrict__ part, int B, int S) {
  constexpr int R = wrows(CIN);
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * 16, co0 = blockIdx.y * 16, slice = blockIdx.z;
  const long long npix = static_cast<long long>(B) * S * S;
  const long long ps = static_cast<long long>(slice) * kSlicePix;
  const int r = r0 + (lane & 15);
  const int tap = r / CIN, ci = r % CIN;
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const bool conv_row = r < 9 * CIN, bias_row = r == 9 * CIN;
  const int co = co0 + (lane & 15);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int kk = 0; kk < kSlicePix; kk += 32) {
    Frag a, w;
    for (int j = 0; j < 8; ++j) {
      const long long p = ps + kk + 8 * (lane >> 4) + j;
      u16 av = 0, gv = 0;
      if (p < npix) {
        if (conv_row) {
          const int b = static_cast<int>(p / (S * S));
          const int q = static_cast<int>(p % (S * S));
          const int yy = q / S + dy, xx = q % S + dx;
          if (yy >= 0 && yy < S && xx >= 0 && xx < S)
            av = in[((static_cast<long long>(b) * S + yy) * S + xx) * CIN + ci];
        } else if (bias_row) {
          av = 0x3F80;  // 1.0
        }
        gv = g[p * COUT + co];
      }
      a.h[j] = av;
      w.h[j] = gv;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, w.v, acc, 0, 0, 0);
  }
  for (int j = 0; j < 4; ++j) {
    const int rr = r0 + 4 * (lane >> 4) + j;
    part[(static_cast<long long>(slice) * R + rr) * COUT + co] = acc[j];
  }
}

// adds the slices in slice order into the float32 gradient in the master
// layout: W[tap][ci][co] (true channel counts) followed by b[co]
template <int CIN, int COUT>
__global__ void wgrad_reduce_k(const float* __restrict__ part, int nslices, int cin, int cout,
                               float* __restrict__ grad) {
  constexpr int R = wrows(CIN);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nw = 9 * cin * cout;
  if (i >= nw + cout) return;
  long long row;
  int co;
  if (i < nw) {
    const int tap = i / (cin * cout), rem = i % (cin * cout);
    row = static_cast<long long>(tap) * CIN + rem / cout;
    co = rem % cout;
  } else {
    row = 9 * CIN;
    co = i - nw;
  }
  float s = 0.f;
  for (int sl = 0; sl < nslices; ++sl) s += part[(static_cast<long long>(sl) * R + row) * COUT + co];
  grad[i] = s;
}

// ------------------------------------------------------------------ loss
// per sample: l = 1 - (p.u)^2 / ((p.p)(u.u)); gradient / B into g [B][S][S][16]
__global__ __launch_bounds__(256) void loss_k(const float* __restrict__ out, const float* __restrict__ lab,
                                              u16* __restrict__ g, float* __restrict__ loss, int B,
                                              int S) {
  const int b = blockIdx.x;
  const long long n = static_cast<long long>(S) * S;
  const float* p = out + static_cast<long long>(b) * n * 16;
  const float* u = lab + static_cast<long long>(b) * n * 6;
  double pu = 0.0, pp = 0.0, uu = 0.0;
  for (long long i = threadIdx.x; i < n * 6; i += 256) {
    const double pv = p[(i / 6) * 16 + i % 6], uv = u[i];
    pu += pv * uv;
    pp += pv * pv;
    uu += uv * uv;
  }
  __shared__ double red[3][256];
  red[0][threadIdx.x] = pu;
  red[1][threadIdx.x] = pp;
  red[2][threadIdx.x] = uu;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  pu = red[0][0];
  pp = red[1][0];
  uu = red[2][0];
  const double l = 1.0 - pu * pu / (pp * uu);
  if (threadIdx.x == 0) loss[b] = static_cast<float>(l);
  const double cu = -2.0 * pu / (pp * uu) / B, cp = 2.0 * pu * pu / (pp * pp * uu) / B;
  u16* gb = g + static_cast<long long>(b) * n * 16;
  for (long long i = threadIdx.x; i < n * 16; i += 256) {
    const long long pix = i / 16;
    const int f = static_cast<int>(i % 16);
    float v = 0.f;
    if (f < 6) v = static_cast<float>(cu * u[pix * 6 + f] + cp * p[pix * 16 + f]);
    gb[i] = to_bf16(v);
  }
}

// ------------------------------------------------------------------ adam
__global__ void adam_k(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float b1t, float b2t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / (1.f - b1t)) / (sqrtf(vi / (1.f - b2t)) + eps);
}

// master W[tap][ci][co] -> forward wt[co][tap * CINP + ci] and input-gradient
// wd[ci][tap' * COUTP + co] = W[8 - tap'][ci][co] (flipped taps, swapped channels)
__global__ void pack_k(const float* __restrict__ W, int cin, int cout, int cinp, int coutp,
                       u16* __restrict__ wt, u16* __restrict__ wd) {
  const int kpf = kpad(cinp), kpd = kpad(coutp);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nf = coutp * kpf, nd = cinp * kpd;
  if (i < nf) {
    const int co = i / kpf, k = i % kpf, tap = k / cinp, ci = k % cinp;
    float v = 0.f;
    if (co < cout && ci < cin && tap < 9) v = W[(tap * cin + ci) * cout + co];
    wt[i] = to_bf16(v);
  } else if (wd && i < nf + nd) {
    const int j = i - nf;
    const int ci = j / kpd, k = j % kpd, tap = k / coutp, co = k % coutp;
    float v = 0.f;
    if (ci < cin && co < cout && tap < 9) v = W[((8 - tap) * cin + ci) * cout + co];
    wd[j] = to_bf16(v);
  }
}

// float32 output [B][S][S][16] -> float64 start vectors [B][6 S^2], 6 (i S + j) + f
__global__ void out_k(const float* __restrict__ out, double* __restrict__ x0, long long npix) {
  const long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
  if (i >= npix * 6) return;
  x0[i] = out[(i / 6) * 16 + i % 6];
}

}  // namespace

struct cond_cnn {
  int max_batch = 0, max_side = 0;
  bool train = false;
  int nparams = 0;
  int off_w[kLayers], off_b[kLayers];
  hipStream_t stream = nullptr;
  // device
  float *w = nullptr, *m = nullptr, *v = nullptr, *g = nullptr, *part = nullptr, *out = nullptr;
  float* loss = nullptr;
  u16 *act[kLayers] = {}, *gz[kLayers] = {};  // act[0] = input, act[l] = output of layer l
  u16 *wt[kLayers] = {}, *wd[kLayers] = {};
  int t = 0;
  std::vector<float> h_loss;
};

namespace {

template <int L>
struct LayerK {
  static constexpr int CIN = kPad[L], COUT = kPad[L + 1];
};

void pack_all(cond_cnn* n) {
  for (int l = 0; l < kLayers; ++l) {
    const int cinp = kPad[l], coutp = kPad[l + 1];
    const int total = coutp * kpad(cinp) + cinp * kpad(coutp);
    pack_k<<<(total + 255) / 256, 256, 0, n->stream>>>(n->w + n->off_w[l], kCh[l], kCh[l + 1], cinp,
                                                        coutp, n->wt[l], n->wd[l]);
  }
}

template <int CIN, int COUT, int EPI>
void conv(cond_cnn* n, const u16* in, const u16* wt, const float* bias, const u16* mask, void* out,
          int B, int S) {
  const long long npix = static_cast<long long>(B) * S * S;
  const unsigned blocks = static_cast<unsigned>((npix + 16 * kConvWaves - 1) / (16 * kConvWaves));
  conv_k<CIN, COUT, EPI><<<blocks, 64 * kConvWaves, 0, n->stream>>>(in, wt, bias, mask, out, B, S);
}

void forward(cond_cnn* n, int B, int S) {
  conv<8, 64, 0>(n, n->act[0], n->wt[0], n->w + n->off_b[0], nullptr, n->act[1], B, S);
  conv<64, 64, 0>(n, n->act[1], n->wt[1], n->w + n->off_b[1], nullptr, n->act[2], B, S);
  conv<64, 64, 0>(n, n->act[2], n->wt[2], n->w + n->off_b[2], nullptr, n->act[3], B, S);
  conv<64, 16, 1>(n, n->act[3], n->wt[3], n->w + n->off_b[3], nullptr, n->out, B, S);
}

template <int CIN, int COUT>
void wgrad(cond_cnn* n, const u16* in, const u16* g, int layer, int B, int S) {
  const long long npix = static_cast<long long>(B) * S * S;
  const int nslices = static_cast<int>((npix + kSlicePix - 1) / kSlicePix);
  dim3 grid(wrows(CIN) / 16, COUT / 16, nslices);
  wgrad_k<CIN, COUT><<<grid, 64, 0, n->stream>>>(in, g, n->part, B, S);
  const int cin = kCh[layer], cout = kCh[layer + 1];
  const int total = 9 * cin * cout + cout;
  wgrad_reduce_k<CIN, COUT><<<(total + 255) / 256, 256, 0, n->stream>>>(
      n->part, nslices, cin, cout, n->g + n->off_w[layer]);
}

// gradients of the mean loss into n->g; per-sample losses into n->loss
void backward(cond_cnn* n, const float* labels, int B, int S) {
  loss_k<<<B, 256, 0, n->stream>>>(n->out, labels, n->gz[3], n->loss, B, S);
  wgrad<64, 16>(n, n->act[3], n->gz[3], 3, B, S);
  conv<16, 64, 2>(n, n->gz[3], n->wd[3], nullptr, n->act[3], n->gz[2], B, S);
  wgrad<64, 64>(n, n->act[2], n->gz[2], 2, B, S);
  conv<64, 64, 2>(n, n->gz[2], n->wd[2], nullptr, n->act[2], n->gz[1], B, S);
  wgrad<64, 64>(n, n->act[1], n->gz[1], 1, B, S);
  conv<64, 64, 2>(n, n->gz[1], n->wd[1], nullptr, n->act[1], n->gz[0], B, S);
  wgrad<8, 64>(n, n->act[0], n->gz[0], 0, B, S);
}

int check_shape(const cond_cnn* n, int B, int S) {
  if (!n) return fail(COND_EINVAL, "null network");
  if (B < 1 || B > n->max_batch || S < 2 || S > n->max_side)
    return fail(COND_EINVAL, "batch or side outside the sizes the network was created for");
  return COND_OK;
}

}  // namespace

extern "C" {

int cond_cnn_param_count(void) {
  int c = 0;
  for (int l = 0; l < kLayers; ++l) c += 9 * kCh[l] * kCh[l + 1] + kCh[l + 1];
  return c;
}

int cond_cnn_create(int32_t max_batch, int32_t max_side, int32_t train, void* stream,
                    cond_cnn_t** out) {
  if (!out || max_batch < 1 || max_side < 2) return fail(COND_EINVAL, "invalid network sizes");
  *out = nullptr;
  auto* n = new (std::nothrow) cond_cnn();
  if (!n) return fail(COND_ENOMEM, "allocation failed");
  n->max_batch = max_batch;
  n->max_side = max_side;
  n->train = train != 0;
  n->stream = static_cast<hipStream_t>(stream);
  int off = 0;
  for (int l = 0; l < kLayers; ++l) {
    n->off_w[l] = off;
    off += 9 * kCh[l] * kCh[l + 1];
    n->off_b[l] = off;
    off += kCh[l + 1];
  }
  n->nparams = off;
  const long long npix = static_cast<long long>(max_batch) * max_side * max_side;
  const long long nslices = (npix + kSlicePix - 1) / kSlicePix;
  auto fl = [&](float** p, long long count) {
    return hipMalloc(reinterpret_cast<void**>(p), static_cast<size_t>(count) * 4);
  };
  auto hf = [&](u16** p, long long count) {
    return hipMalloc(reinterpret_cast<void**>(p), static_cast<size_t>(count) * 2);
  };
  hipError_t e = hipSuccess;
  e = fl(&n->w, n->nparams);
  if (e == hipSuccess) e = fl(&n->out, npix * 16);
  for (int l = 0; l < kLayers && e == hipSuccess; ++l) {
    e = hf(&n->act[l], npix * kPad[l]);
    if (e == hipSuccess) e = hf(&n->wt[l], static_cast<long long>(kPad[l + 1]) * kpad(kPad[l]));
  }
  if (n->train) {
    for (float** p : {&n->m, &n->v, &n->g})
      if (e == hipSuccess) e = fl(p, n->nparams);
    if (e == hipSuccess) e = fl(&n->part, nslices * wrows(64) * 64);
    if (e == hipSuccess) e = fl(&n->loss, max_batch);
    for (int l = 0; l < kLayers && e == hipSuccess; ++l) {
      e = hf(&n->gz[l], npix * kPad[l + 1]);
      if (e == hipSuccess) e = hf(&n->wd[l], static_cast<long long>(kPad[l]) * kpad(kPad[l + 1]));
    }
  }
  if (e != hipSuccess) {
    cond_cnn_destroy(n);
    return fail(COND_EHIP, std::string("cnn allocation: ") + hipGetErrorString(e));
  }
  *out = n;
  return COND_OK;
}

void cond_cnn_destroy(cond_cnn_t* n) {
  if (!n) return;
  if (n->stream) hipStreamSynchronize(n->stream);
  for (float* p : {n->w, n->m, n->v, n->g, n->part, n->out, n->loss})
    if (p) hipFree(p);
  for (int l = 0; l < kLayers; ++l)
    for (u16* p : {n->act[l], n->gz[l], n->wt[l], n->wd[l]})
      if (p) hipFree(p);
  delete n;
}

int cond_cnn_set_params(cond_cnn_t* n, const float* params) {
  if (!n || !params) return fail(COND_EINVAL, "null argument");
  NCHK(hipMemcpyAsync(n->w, params, n->nparams * 4, hipMemcpyHostToDevice, n->stream));
  if (n->train) {
    NCHK(hipMemsetAsync(n->m, 0, n->nparams * 4, n->stream));
    NCHK(hipMemsetAsync(n->v, 0, n->nparams * 4, n->stream));
  }
  n->t = 0;
  pack_all(n);
  NCHK(hipStreamSynchronize(n->stream));
  return COND_OK;
}

int cond_cnn_get_params(const cond_cnn_t* n, float* params) {
  if (!n || !params) return fail(COND_EINVAL, "null argument");
  NCHK(hipMemcpyAsync(params, n->w, n->nparams * 4, hipMemcpyDeviceToHost, n->stream));
  NCHK(hipStreamSynchronize(n->stream));
  return COND_OK;
}

int cond_cnn_predict(cond_cnn_t* n, const double* cells, int32_t batch, int32_t side, double* x0) {
  int st = check_shape(n, batch, side);
  if (st) return st;
  if (!cells || !x0) return fail(COND_EINVAL, "null argument");
  const long long npix = static_cast<long long>(batch) * side * side;
  prep_k<<<static_cast<unsigned>((npix + 255) / 256), 256, 0, n->stream>>>(cells, n->act[0], batch, side);
  forward(n, batch, side);
  out_k<<<static_cast<unsigned>((npix * 6 + 255) / 256), 256, 0, n->stream>>>(n->out, x0, npix);
  NCHK(hipGetLastError());
  NCHK(hipStreamSynchronize(n->stream));
  return COND_OK;
}

int cond_cnn_gradients(cond_cnn_t* n, const double* cells, const float* labels, int32_t batch,
                       int32_t side, float* grad, float* losses) {
  int st = check_shape(n, batch, side);
  if (st) return st;
  if (!n->train) return fail(COND_ESTATE, "network was created without training buffers");
  if (!cells || !labels) return fail(COND_EINVAL, "null argument");
  const long long npix = static_cast<long long>(batch) * side * side;
  prep_k<<<static_cast<unsigned>((npix + 255) / 256), 256, 0, n->stream>>>(cells, n->act[0], batch, side);
  forward(n, batch, side);
  backward(n, labels, batch, side);
  NCHK(hipGetLastError());
  if (grad) NCHK(hipMemcpyAsync(grad, n->g, n->nparams * 4, hipMemcpyDeviceToHost, n->stream));
  if (losses) NCHK(hipMemcpyAsync(losses, n->loss, batch * 4, hipMemcpyDeviceToHost, n->stream));
  NCHK(hipStreamSynchronize(n->stream));
  return COND_OK;
}

int cond_cnn_train_step(cond_cnn_t* n, const double* cells, const float* labels, int32_t batch,
                        int32_t side, float lr, float* mean_loss) {
  int st = check_shape(n, batch, side);
  if (st) return st;
  if (!n->train) return fail(COND_ESTATE, "network was created without training buffers");
  if (!cells || !labels || !(lr > 0.f)) return fail(COND_EINVAL, "invalid argument");
  const long long npix = static_cast<long long>(batch) * side * side;
  prep_k<<<static_cast<unsigned>((npix + 255) / 256), 256, 0, n->stream>>>(cells, n->act[0], batch, side);
  forward(n, batch, side);
  backward(n, labels, batch, side);
  n->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float b1t = std::pow(b1, static_cast<float>(n->t)), b2t = std::pow(b2, static_cast<float>(n->t));
  adam_k<<<(n->nparams + 255) / 256, 256, 0, n->stream>>>(n->w, n->g, n->m, n->v, n->nparams, lr, b1,
                                                          b2, 1e-8f, b1t, b2t);
  pack_all(n);
  NCHK(hipGetLastError());
  if (mean_loss) {
    n->h_loss.resize(batch);
    NCHK(hipMemcpyAsync(n->h_loss.data(), n->loss, batch * 4, hipMemcpyDeviceToHost, n->stream));
    NCHK(hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (float l : n->h_loss) s += l;
    *mean_loss = static_cast<float>(s / batch);
  }
  return COND_OK;
}

int cond_cnn_activation(const cond_cnn_t* n, int32_t layer, int32_t batch, int32_t side, float* host) {
  int st = check_shape(n, batch, side);
  if (st) return st;
  if (!host || layer < 0 || layer > kLayers) return fail(COND_EINVAL, "invalid argument");
  const long long npix = static_cast<long long>(batch) * side * side;
  if (layer == kLayers) {
    NCHK(hipMemcpyAsync(host, n->out, npix * 16 * 4, hipMemcpyDeviceToHost, n->stream));
    NCHK(hipStreamSynchronize(n->stream));
    return COND_OK;
  }
  std::vector<u16> tmp(static_cast<size_t>(npix) * kPad[layer]);
  NCHK(hipMemcpyAsync(tmp.data(), n->act[layer], tmp.size() * 2, hipMemcpyDeviceToHost, n->stream));
  NCHK(hipStreamSynchronize(n->stream));
  for (size_t i = 0; i < tmp.size(); ++i) {
    const unsigned u = static_cast<unsigned>(tmp[i]) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    host[i] = f;
  }
  return COND_OK;
}

}  // extern "C"
