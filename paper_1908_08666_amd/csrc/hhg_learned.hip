// Learned 3x3 block smoother: node features, network inference on the matrix
// cores, training (forward, backward and Adam on the device), training-record
// collection and the preconditioner blocks P = (I + M)^T D^{-1} (I + M).
//
// Not in the paper (its smoother is Gauss-Seidel inside multigrid); the
// features are the coefficient on the 15-point stencil patch of Sec. 2.4.
//
// Inference: one wavefront evaluates 16 records per step with the layers
// transposed, H^T = W1^T F^T and O^T = W2^T H^T, so that the accumulator
// layout of the first product (lane l: rows 4(l/16)..+3 of column l%16) is
// exactly the B-operand layout of the second and no data moves between the
// two: per 16 records 4 + 4 MFMA 16x16x16 BF16 -> FP32 instructions, the
// weights held in registers for the whole launch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "hhg_device.h"

struct hhg_mlp_ctx {
  int device = -1;
  float *buf = nullptr;       // one allocation: w, m, v, w2r, then the BF16 tables
  float *w = nullptr;         // FP32 master parameters [NPARAM]
  float *m = nullptr, *v = nullptr;   // Adam moments
  float *w2r = nullptr;       // W2 after BF16 rounding, FP32 [64][9] (backward)
  uint16_t *w1t = nullptr;    // BF16 [64][16]: w1t[j][i] = W1[i][j]
  uint16_t *w2t = nullptr;    // BF16 [16][64]: w2t[o][j] = W2[j][o], rows o >= 9 zero
  int64_t step = 0;
};

namespace hhg {

int diag_blocks(hhg_ctx *h, const double *k, int method, double *D, hipStream_t st);

namespace {

constexpr int NIN = HHG_MLP_IN, NHID = HHG_MLP_HIDDEN, NOUT = HHG_MLP_OUT;
constexpr int NPARAM = HHG_MLP_NPARAM;
constexpr int OFF_B1 = NIN * NHID;                 // 1024
constexpr int OFF_W2 = OFF_B1 + NHID;              // 1088
constexpr int OFF_B2 = OFF_W2 + NHID * NOUT;       // 1664
constexpr int REC_U16 = HHG_SAMPLE_BYTES / 2;      // record stride in uint16
constexpr int REC_F32 = 8;                         // first float of a record (after 32 B)

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs)
__host__ __device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_val(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// ---------------------------------------------------------------- features
__device__ __forceinline__ int plane_base_l(int n, int k) {
  const int a = n + 1, b = n + 1 - k;
  return a * (a + 1) * (a + 2) / 6 - b * (b + 1) * (b + 2) / 6;
}

// (i, j, k) of local slot ls of a macro with n intervals
__device__ __forceinline__ void local_ijk(int n, int ls, int &i, int &j, int &k) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (plane_base_l(n, mid) <= ls) lo = mid; else hi = mid - 1;
  }
  k = lo;
  const int pos = ls - plane_base_l(n, k);
  const int s = tri_root_dev(pos);
  i = pos - s * (s + 1) / 2;
  j = s - i;
}

// 16 BF16 features of the node copy (i, j, k) of macro mi (K: the macro's
// coefficient slots)
__device__ __forceinline__ void node_features(const MacroInfo &mi, const double *__restrict__ K,
                                              int i, int j, int k, uint16_t *out) {
  const int n = mi.n;
  const double kc = K[plane_base_l(n, k) + (i + j) * (i + j + 1) / 2 + i];
  double v[15];
  v[0] = kc;
#pragma unroll
  for (int d = 0; d < NDIR; ++d) {
    const int a = i + DIR_I[d], b = j + DIR_J[d], c = k + DIR_K[d];
    double val = kc;
    if (a >= 0 && b >= 0 && c >= 0 && a + b + c <= n) {
      const int z = zero_set(a, b, c, n);
      val = ((mi.dmask >> z) & 1u) ? 0.0 : K[plane_base_l(n, c) + (a + b) * (a + b + 1) / 2 + a];
    }
    v[1 + d] = val;
  }
  double total = v[0];
#pragma unroll
  for (int q = 1; q < 15; ++q) total += v[q];
  const double mean = total / 15.0;
#pragma unroll
  for (int q = 0; q < 15; ++q) out[q] = bf16_rne((float)(v[q] / mean));
  out[15] = bf16_rne((float)((double)mi.level / 8.0));
}

__global__ __launch_bounds__(256) void k_features(const MacroInfo *__restrict__ minfo,
                                                  const double *__restrict__ kc,
                                                  uint16_t *__restrict__ feat) {
  const int m = blockIdx.y;
  const MacroInfo mi = minfo[m];
  const int ls = blockIdx.x * blockDim.x + threadIdx.x;
  if (ls >= (int)macro_nodes(mi.n)) return;
  int i, j, k;
  local_ijk(mi.n, ls, i, j, k);
  uint16_t f[16];
  node_features(mi, kc + mi.off, i, j, k, f);
  uint2 *dst = reinterpret_cast<uint2 *>(feat + (mi.off + ls) * 16);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    dst[q] = make_uint2((uint32_t)f[4 * q] | ((uint32_t)f[4 * q + 1] << 16),
                        (uint32_t)f[4 * q + 2] | ((uint32_t)f[4 * q + 3] << 16));
}

// --------------------------------------------------------------- inference
// out[q][0..8] = W2^T relu(W1^T f_q + b1)_bf16 + b2 for records q < n;
// hid (optional): the BF16 hidden layer [n][64].
__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t *__restrict__ feat,
                                                     int64_t stride, int64_t n,
                                                     const uint16_t *__restrict__ w1t,
                                                     const uint16_t *__restrict__ w2t,
                                                     const float *__restrict__ w,
                                                     float *__restrict__ out,
                                                     uint16_t *__restrict__ hid) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int col = lane & 15, kb = lane >> 4;
  v4s a1[4], a2[4];
  float bias1[4][4], bias2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint2 p1 = *reinterpret_cast<const uint2 *>(w1t + (16 * t + col) * 16 + 4 * kb);
    const uint2 p2 = *reinterpret_cast<const uint2 *>(w2t + col * 64 + 16 * t + 4 * kb);
    a1[t] = v4s{(short)(p1.x & 0xFFFF), (short)(p1.x >> 16), (short)(p1.y & 0xFFFF), (short)(p1.y >> 16)};
    a2[t] = v4s{(short)(p2.x & 0xFFFF), (short)(p2.x >> 16), (short)(p2.y & 0xFFFF), (short)(p2.y >> 16)};
#pragma unroll
    for (int q = 0; q < 4; ++q) bias1[t][q] = w[OFF_B1 + 16 * t + 4 * kb + q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) bias2[q] = (4 * kb + q < NOUT) ? w[OFF_B2 + 4 * kb + q] : 0.0f;

  for (int64_t tile = wave; tile * 16 < n; tile += nwaves) {
    const int64_t rec = tile * 16 + col;
    v4s bf = {0, 0, 0, 0};
    if (rec < n) {
      const uint2 pf = *reinterpret_cast<const uint2 *>(feat + rec * stride + 4 * kb);
      bf = v4s{(short)(pf.x & 0xFFFF), (short)(pf.x >> 16), (short)(pf.y & 0xFFFF), (short)(pf.y >> 16)};
    }
    v4s bh[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      v4f acc = {bias1[t][0], bias1[t][1], bias1[t][2], bias1[t][3]};
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[t], bf, acc, 0, 0, 0);
      uint16_t hb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) hb[q] = bf16_rne(fmaxf(acc[q], 0.0f));
      bh[t] = v4s{(short)hb[0], (short)hb[1], (short)hb[2], (short)hb[3]};
      if (hid && rec < n)
        *reinterpret_cast<uint2 *>(hid + rec * NHID + 16 * t + 4 * kb) =
            make_uint2((uint32_t)hb[0] | ((uint32_t)hb[1] << 16),
                       (uint32_t)hb[2] | ((uint32_t)hb[3] << 16));
    }
    v4f o = {bias2[0], bias2[1], bias2[2], bias2[3]};
#pragma unroll
    for (int t = 0; t < 4; ++t) o = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[t], bh[t], o, 0, 0, 0);
    if (rec < n) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * kb + q < NOUT) out[rec * NOUT + 4 * kb + q] = o[q];
    }
  }
}

// BF16 copies of the master weights in the inference layouts
__global__ void k_pack_weights(const float *__restrict__ w, uint16_t *__restrict__ w1t,
                               uint16_t *__restrict__ w2t, float *__restrict__ w2r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < NIN * NHID) {
    const int i = t / NHID, j = t % NHID;
    w1t[j * NIN + i] = bf16_rne(w[t]);
  } else if (t < NIN * NHID + 16 * NHID) {
    const int q = t - NIN * NHID;
    const int o = q / NHID, j = q % NHID;
    if (o < NOUT) {
      const uint16_t b = bf16_rne(w[OFF_W2 + j * NOUT + o]);
      w2t[o * NHID + j] = b;
      w2r[j * NOUT + o] = bf16_val(b);
    } else {
      w2t[o * NHID + j] = 0;
    }
  }
}

// ---------------------------------------------------------------- training
// Per record of a batch of B: loss, output gradient d2 = dl/do (9, padded to
// 16) and hidden gradient dz1 (64); per-block partial loss sums.
__global__ __launch_bounds__(256) void k_train_record(const uint16_t *__restrict__ rec,
                                                      int64_t B, const float *__restrict__ out,
                                                      const uint16_t *__restrict__ hid,
                                                      const float *__restrict__ w2r,
                                                      float *__restrict__ d2,
                                                      float *__restrict__ dz1,
                                                      double *__restrict__ part) {
  __shared__ double sh[4];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double loss = 0.0;
  if (s < B) {
    const float *val = reinterpret_cast<const float *>(rec + s * REC_U16) + REC_F32;
    const float r[3] = {val[0], val[1], val[2]};
    const float e[3] = {val[3], val[4], val[5]};
    const float S[3][3] = {{val[6], val[9], val[10]}, {val[9], val[7], val[11]},
                           {val[10], val[11], val[8]}};
    float G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) G[a][b] = out[s * NOUT + 3 * a + b] + (a == b ? 1.0f : 0.0f);
    float u[3], v[3], z[3], dz[3], dv[3], du[3];
    const float inv2 = 2.0f / (float)B;
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = G[a][0] * r[0] + G[a][1] * r[1] + G[a][2] * r[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = S[a][0] * u[0] + S[a][1] * u[1] + S[a][2] * u[2];
#pragma unroll
    for (int b = 0; b < 3; ++b) z[b] = G[0][b] * v[0] + G[1][b] * v[1] + G[2][b] * v[2];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const float d = z[b] - e[b];
      loss += (double)d * d;
      dz[b] = inv2 * d;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) dv[a] = G[a][0] * dz[0] + G[a][1] * dz[1] + G[a][2] * dz[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) du[a] = S[a][0] * dv[0] + S[a][1] * dv[1] + S[a][2] * dv[2];
    float g2[NOUT];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) g2[3 * a + b] = v[a] * dz[b] + du[a] * r[b];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) d2[s * 16 + o] = g2[o];
    for (int j = 0; j < NHID; ++j) {
      float dh = 0.0f;
#pragma unroll
      for (int o = 0; o < NOUT; ++o) dh = fmaf(w2r[j * NOUT + o], g2[o], dh);
      dz1[s * NHID + j] = bf16_val(hid[s * NHID + j]) > 0.0f ? dh : 0.0f;
    }
  }
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_down(loss, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = loss;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Gradient partial sums of one chunk of GCHUNK records, one workgroup per
// chunk: the chunk's features, hidden activations and gradients are staged in
// LDS, then each thread sums its parameters over the chunk's records in
// FP64 (products of FP32 values are exact in FP64).  Parameter p of chunk c
// goes to gpart[c * NPARAM + p].
constexpr int GCHUNK = 64;
__global__ __launch_bounds__(256) void k_grad_part(const uint16_t *__restrict__ rec, int64_t B,
                                                   const uint16_t *__restrict__ hid,
                                                   const float *__restrict__ d2,
                                                   const float *__restrict__ dz1,
                                                   double *__restrict__ gpart) {
  __shared__ float sf[GCHUNK][NIN];
  __shared__ float sdz[GCHUNK][NHID];
  __shared__ float shd[GCHUNK][NHID];
  __shared__ float sd2[GCHUNK][NOUT];
  const int64_t s0 = (int64_t)blockIdx.x * GCHUNK;
  const int cnt = (int)min((int64_t)GCHUNK, B - s0);
  for (int t = threadIdx.x; t < GCHUNK * NIN; t += blockDim.x) {
    const int r = t / NIN, i = t % NIN;
    sf[r][i] = r < cnt ? bf16_val(rec[(s0 + r) * REC_U16 + i]) : 0.0f;
  }
  for (int t = threadIdx.x; t < GCHUNK * NHID; t += blockDim.x) {
    const int r = t / NHID, j = t % NHID;
    sdz[r][j] = r < cnt ? dz1[(s0 + r) * NHID + j] : 0.0f;
    shd[r][j] = r < cnt ? bf16_val(hid[(s0 + r) * NHID + j]) : 0.0f;
  }
  for (int t = threadIdx.x; t < GCHUNK * NOUT; t += blockDim.x) {
    const int r = t / NOUT, o = t % NOUT;
    sd2[r][o] = r < cnt ? d2[(s0 + r) * 16 + o] : 0.0f;
  }
  __syncthreads();
  for (int p = threadIdx.x; p < NPARAM; p += blockDim.x) {
    double g = 0.0;
    if (p < OFF_B1) {
      const int i = p / NHID, j = p % NHID;
      for (int r = 0; r < cnt; ++r) g += (double)sf[r][i] * (double)sdz[r][j];
    } else if (p < OFF_W2) {
      const int j = p - OFF_B1;
      for (int r = 0; r < cnt; ++r) g += (double)sdz[r][j];
    } else if (p < OFF_B2) {
      const int q = p - OFF_W2, j = q / NOUT, o = q % NOUT;
      for (int r = 0; r < cnt; ++r) g += (double)shd[r][j] * (double)sd2[r][o];
    } else {
      const int o = p - OFF_B2;
      for (int r = 0; r < cnt; ++r) g += (double)sd2[r][o];
    }
    gpart[(int64_t)blockIdx.x * NPARAM + p] = g;
  }
}

// One thread per parameter: the chunk partials summed in chunk order (FP64),
// then either stored (grad != null) or applied by an Adam step.  Thread 0
// also sums the loss partials of the batch into loss_out.
__global__ __launch_bounds__(256) void k_grad_adam(const double *__restrict__ gpart, int nchunk,
                                                   int64_t B, const double *__restrict__ part,
                                                   int npart, double *__restrict__ loss_out,
                                                   float *__restrict__ grad, float *__restrict__ w,
                                                   float *__restrict__ mom1, float *__restrict__ mom2,
                                                   float lr, float beta1, float beta2, float eps,
                                                   float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0) {
    double l = 0.0;
    for (int q = 0; q < npart; ++q) l += part[q];
    *loss_out = l / (double)B;
  }
  if (p >= NPARAM) return;
  double g = 0.0;
  for (int c = 0; c < nchunk; ++c) g += gpart[(int64_t)c * NPARAM + p];
  const float gf = (float)g;
  if (grad) {
    grad[p] = gf;
    return;
  }
  const float m = beta1 * mom1[p] + (1.0f - beta1) * gf;
  const float v = beta2 * mom2[p] + (1.0f - beta2) * gf * gf;
  mom1[p] = m;
  mom2[p] = v;
  w[p] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// ------------------------------------------------------ record collection
__device__ __forceinline__ void inv_sym3(const double *d, double *o) {
  // d = xx yy zz xy xz yz; o likewise
  const double a = d[0], b = d[1], c = d[2], x = d[3], y = d[4], z = d[5];
  const double A = b * c - z * z, Bc = y * z - x * c, C = x * z - b * y;
  const double r = 1.0 / (a * A + x * Bc + y * C);
  o[0] = A * r;
  o[1] = (a * c - y * y) * r;
  o[2] = (a * b - x * x) * r;
  o[3] = Bc * r;
  o[4] = C * r;
  o[5] = (x * y - a * z) * r;
}

__global__ __launch_bounds__(256) void k_collect(const MacroInfo *__restrict__ minfo, int n_macro,
                                                 const double *__restrict__ kc,
                                                 const double *__restrict__ r,
                                                 const double *__restrict__ e,
                                                 const double *__restrict__ D, int64_t N,
                                                 const int64_t *__restrict__ slots, int64_t n,
                                                 uint16_t *__restrict__ rec) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int64_t slot = slots[q];
  int lo = 0, hi = n_macro - 1;   // macro: largest m with off <= slot
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (minfo[mid].off <= slot) lo = mid; else hi = mid - 1;
  }
  const MacroInfo mi = minfo[lo];
  int i, j, k;
  local_ijk(mi.n, (int)(slot - mi.off), i, j, k);
  uint16_t f[16];
  node_features(mi, kc + mi.off, i, j, k, f);
  uint16_t *dst = rec + q * REC_U16;
#pragma unroll
  for (int c = 0; c < 16; ++c) dst[c] = f[c];
  double d6[6], di[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) d6[c] = D[c * N + slot];
  inv_sym3(d6, di);
  const double t = (d6[0] + d6[1] + d6[2]) / 3.0;
  const double rv[3] = {r[slot], r[N + slot], r[2 * N + slot]};
  const double w0 = di[0] * rv[0] + di[3] * rv[1] + di[4] * rv[2];
  const double w1 = di[3] * rv[0] + di[1] * rv[1] + di[5] * rv[2];
  const double w2 = di[4] * rv[0] + di[5] * rv[1] + di[2] * rv[2];
  const double ev[3] = {e[slot], e[N + slot], e[2 * N + slot]};
  const double s = sqrt((w0 * w0 + w1 * w1 + w2 * w2) + (ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]));
  float *val = reinterpret_cast<float *>(dst) + REC_F32;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    val[c] = (float)(rv[c] / (t * s));
    val[3 + c] = (float)(ev[c] / s);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) val[6 + c] = (float)(t * di[c]);
#pragma unroll
  for (int c = 12; c < 24; ++c) val[c] = 0.0f;
}

// ---------------------------------------------------- preconditioner blocks
// mean of the network output over the copies of every interface node
__global__ void k_group_avg9(const int64_t *__restrict__ ptr, const int64_t *__restrict__ slots,
                             int64_t ng, float *__restrict__ mout) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = t / NOUT;
  const int c = (int)(t - NOUT * g);
  if (g >= ng) return;
  double sum = 0.0;
  const int64_t a = ptr[g], b = ptr[g + 1];
  for (int64_t q = a; q < b; ++q) sum += mout[slots[q] * NOUT + c];
  const float avg = (float)(sum / (double)(b - a));
  for (int64_t q = a; q < b; ++q) mout[slots[q] * NOUT + c] = avg;
}

// P <- (I + M)^T P (I + M) at every non-Dirichlet slot (P holds D^{-1})
__global__ void k_learned_blocks(double *__restrict__ P, const float *__restrict__ mout,
                                 const uint8_t *__restrict__ fl, int64_t N) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N;
       s += (int64_t)gridDim.x * blockDim.x) {
    if (fl[s] & 1) continue;
    double G[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) G[a][b] = (double)mout[s * NOUT + 3 * a + b] + (a == b ? 1.0 : 0.0);
    const double Di[3][3] = {{P[s], P[3 * N + s], P[4 * N + s]},
                             {P[3 * N + s], P[N + s], P[5 * N + s]},
                             {P[4 * N + s], P[5 * N + s], P[2 * N + s]}};
    double T[3][3];   // D^{-1} G
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) T[a][c] = Di[a][0] * G[0][c] + Di[a][1] * G[1][c] + Di[a][2] * G[2][c];
    double R[3][3];   // G^T D^{-1} G
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) R[a][c] = G[0][a] * T[0][c] + G[1][a] * T[1][c] + G[2][a] * T[2][c];
    P[s] = R[0][0];
    P[N + s] = R[1][1];
    P[2 * N + s] = R[2][2];
    P[3 * N + s] = 0.5 * (R[0][1] + R[1][0]);
    P[4 * N + s] = 0.5 * (R[0][2] + R[2][0]);
    P[5 * N + s] = 0.5 * (R[1][2] + R[2][1]);
  }
}

dim3 fwd_grid(int64_t n) {
  const int64_t tiles = (n + 15) / 16;
  const int64_t blocks = (tiles + 3) / 4;
  return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 8192)));
}

int check_model(hhg_mlp m) {
  if (!m || !m->buf) return fail(HHG_EINVAL, "null model");
  int dev = -1;
  HHG_HIP(hipGetDevice(&dev));
  if (dev != m->device) return fail(HHG_EINVAL, "model lives on another device");
  return HHG_OK;
}

int launch_forward(hhg_mlp m, const uint16_t *feat, int64_t stride, int64_t n, float *out,
                   uint16_t *hid, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_forward, fwd_grid(n), dim3(256), 0, st, feat, stride, n, m->w1t, m->w2t,
                     m->w, out, hid);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

int pack(hhg_mlp m, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_weights, dim3((NIN * NHID + 16 * NHID + 255) / 256), dim3(256), 0, st,
                     m->w, m->w1t, m->w2t, m->w2r);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

// Scratch of one training batch.
struct TrainScratch {
  void *buf = nullptr;
  float *out = nullptr, *d2 = nullptr, *dz1 = nullptr;
  uint16_t *hid = nullptr;
  double *part = nullptr, *loss = nullptr, *gpart = nullptr;
  int nblk = 0;
  ~TrainScratch() {
    if (buf) (void)hipFree(buf);
  }
  int alloc(int64_t B, int64_t nloss) {
    nblk = (int)((B + 255) / 256);
    const size_t a = 256;
    auto up = [&](size_t v) { return (v + a - 1) / a * a; };
    const size_t s_out = up(B * NOUT * 4), s_d2 = up(B * 16 * 4), s_dz = up(B * NHID * 4);
    const size_t s_hid = up(B * NHID * 2), s_part = up(nblk * 8), s_loss = up(nloss * 8);
    const size_t s_gpart = up((size_t)((B + GCHUNK - 1) / GCHUNK) * NPARAM * 8);
    HHG_HIP(hipMalloc(&buf, s_out + s_d2 + s_dz + s_hid + s_part + s_loss + s_gpart));
    char *p = static_cast<char *>(buf);
    out = reinterpret_cast<float *>(p);
    p += s_out;
    d2 = reinterpret_cast<float *>(p);
    p += s_d2;
    dz1 = reinterpret_cast<float *>(p);
    p += s_dz;
    hid = reinterpret_cast<uint16_t *>(p);
    p += s_hid;
    part = reinterpret_cast<double *>(p);
    p += s_part;
    loss = reinterpret_cast<double *>(p);
    p += s_loss;
    gpart = reinterpret_cast<double *>(p);
    return HHG_OK;
  }
};

// forward + per-record backward + gradient (grad != null) or Adam step
int train_batch(hhg_mlp m, const uint16_t *rec, int64_t B, TrainScratch &ts, double *loss_out,
                float *grad, const hhg_train_opts *o, hipStream_t st) {
  int rc = launch_forward(m, rec, REC_U16, B, ts.out, ts.hid, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_train_record, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, rec, B,
                     ts.out, ts.hid, m->w2r, ts.d2, ts.dz1, ts.part);
  float c1 = 1.0f, c2 = 1.0f, lr = 0.0f, b1 = 0.0f, b2 = 0.0f, eps = 0.0f;
  if (!grad) {
    ++m->step;
    c1 = (float)(1.0 / (1.0 - std::pow((double)o->beta1, (double)m->step)));
    c2 = (float)(1.0 / (1.0 - std::pow((double)o->beta2, (double)m->step)));
    lr = o->lr;
    b1 = o->beta1;
    b2 = o->beta2;
    eps = o->eps;
  }
  const int npart = (int)((B + 255) / 256);   // partials written for this batch
  const int nchunk = (int)((B + GCHUNK - 1) / GCHUNK);
  hipLaunchKernelGGL(k_grad_part, dim3(nchunk), dim3(256), 0, st, rec, B, ts.hid, ts.d2, ts.dz1,
                     ts.gpart);
  hipLaunchKernelGGL(k_grad_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, ts.gpart, nchunk, B,
                     ts.part, npart, loss_out, grad, m->w, m->m, m->v, lr, b1, b2, eps, c1, c2);
  HHG_HIP(hipGetLastError());
  if (!grad) return pack(m, st);
  return HHG_OK;
}

bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

}  // namespace

// Learned preconditioner blocks for a solve: P holds D^{-1} on entry.
int learned_precond(hhg_ctx *h, const double *k, double *P, uint16_t *feat, float *mout,
                    hipStream_t st) {
  hhg_mlp m = h->model;
  int rc = check_model(m);
  if (rc) return rc;
  const int64_t N = h->n_nodes;
  {
    ProfScope ps(h, HHG_K_LEARNED, st);
    int maxn = 0;
    for (auto &mi : h->minfo) maxn = std::max(maxn, (int)macro_nodes(mi.n));
    hipLaunchKernelGGL(k_features, dim3((maxn + 255) / 256, h->n_macro), dim3(256), 0, st,
                       h->d_minfo, k, feat);
    if ((rc = launch_forward(m, feat, 16, N, mout, nullptr, st))) return rc;
  }
  if (h->n_grp > 0)
    hipLaunchKernelGGL(k_group_avg9, dim3((unsigned)((NOUT * h->n_grp + 255) / 256)), dim3(256), 0,
                       st, h->d_grp_ptr, h->d_grp_slot, h->n_grp, mout);
  const int64_t blocks = std::min<int64_t>((N + 255) / 256, 4096);
  hipLaunchKernelGGL(k_learned_blocks, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st,
                     P, mout, h->d_flags, N);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

}  // namespace hhg

using namespace hhg;

extern "C" {

int hhg_mlp_create(hhg_mlp *out) {
  if (!out) return fail(HHG_EINVAL, "null output");
  *out = nullptr;
  auto *m = new (std::nothrow) hhg_mlp_ctx();
  if (!m) return fail(HHG_EINVAL, "out of host memory");
  hipError_t e = hipGetDevice(&m->device);
  const size_t nf = 3 * (size_t)NPARAM + NHID * NOUT;      // w, m, v, w2r
  const size_t bytes = ((nf * 4 + 255) / 256) * 256 + (NIN * NHID + 16 * NHID) * 2;
  if (e == hipSuccess) e = hipMalloc((void **)&m->buf, bytes);
  if (e == hipSuccess) e = hipMemset(m->buf, 0, bytes);
  if (e != hipSuccess) {
    if (m->buf) (void)hipFree(m->buf);
    delete m;
    return hip_fail(e, "hhg_mlp_create");
  }
  m->w = m->buf;
  m->m = m->w + NPARAM;
  m->v = m->m + NPARAM;
  m->w2r = m->v + NPARAM;
  m->w1t = reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(m->buf) + ((nf * 4 + 255) / 256) * 256);
  m->w2t = m->w1t + NIN * NHID;
  *out = m;
  return HHG_OK;
}

int hhg_mlp_destroy(hhg_mlp m) {
  if (!m) return HHG_OK;
  if (m->buf) (void)hipFree(m->buf);
  delete m;
  return HHG_OK;
}

int hhg_mlp_set_weights(hhg_mlp m, const float *w) {
  int rc = check_model(m);
  if (rc) return rc;
  if (!w) return fail(HHG_EINVAL, "null weights");
  for (int p = 0; p < NPARAM; ++p)
    if (!std::isfinite(w[p])) return fail(HHG_EINVAL, "non-finite weight");
  HHG_HIP(hipMemcpy(m->w, w, NPARAM * sizeof(float), hipMemcpyHostToDevice));
  HHG_HIP(hipMemset(m->m, 0, 2 * NPARAM * sizeof(float)));
  m->step = 0;
  if ((rc = pack(m, nullptr))) return rc;
  HHG_HIP(hipDeviceSynchronize());
  return HHG_OK;
}

int hhg_mlp_get_weights(hhg_mlp m, float *w) {
  int rc = check_model(m);
  if (rc) return rc;
  if (!w) return fail(HHG_EINVAL, "null weights");
  HHG_HIP(hipDeviceSynchronize());
  HHG_HIP(hipMemcpy(w, m->w, NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  return HHG_OK;
}

int hhg_learn_features(hhg_handle h, const double *k, uint16_t *feat, void *stream) {
  if (!h || !k || !feat) return fail(HHG_EINVAL, "null argument");
  if (!aligned(k, 8) || !aligned(feat, 8)) return fail(HHG_EINVAL, "misaligned pointer");
  int rc = ensure_device(h);
  if (rc) return rc;
  int maxn = 0;
  for (auto &mi : h->minfo) maxn = std::max(maxn, (int)macro_nodes(mi.n));
  ProfScope ps(h, HHG_K_LEARNED, (hipStream_t)stream);
  hipLaunchKernelGGL(k_features, dim3((maxn + 255) / 256, h->n_macro), dim3(256), 0,
                     (hipStream_t)stream, h->d_minfo, k, feat);
  HHG_HIP(hipGetLastError());
  return HHG_OK;
}

int hhg_mlp_forward(hhg_mlp m, const uint16_t *feat, int64_t stride, int64_t n, float *out,
                    void *stream) {
  int rc = check_model(m);
  if (rc) return rc;
  if (!feat || !out) return fail(HHG_EINVAL, "null argument");
  if (n < 0 || stride < 16 || stride % 4) return fail(HHG_EINVAL, "bad record count or stride");
  if (!aligned(feat, 8) || !aligned(out, 4)) return fail(HHG_EINVAL, "misaligned pointer");
  if (n == 0) return HHG_OK;
  return launch_forward(m, feat, stride, n, out, nullptr, (hipStream_t)stream);
}

int hhg_learn_collect(hhg_handle h, int32_t method, const double *k, const double *r,
                      const double *e, const int64_t *slots, int64_t n, void *samples,
                      void *stream) {
  if (!h || !k || !r || !e || !slots || !samples) return fail(HHG_EINVAL, "null argument");
  if (n < 1) return fail(HHG_EINVAL, "n must be >= 1");
  if (method != HHG_METHOD_SCALED && method != HHG_METHOD_ONTHEFLY)
    return fail(HHG_EINVAL, "unknown operator method");
  if (!aligned(samples, 16) || !aligned(k, 8) || !aligned(r, 8) || !aligned(e, 8) ||
      !aligned(slots, 8))
    return fail(HHG_EINVAL, "misaligned pointer");
  int rc = ensure_device(h);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = h->n_nodes;
  {
    // the kernel indexes by these slots: check them on the host first
    std::vector<int64_t> hs((size_t)n);
    HHG_HIP(hipMemcpyAsync(hs.data(), slots, n * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HHG_HIP(hipStreamSynchronize(st));
    for (int64_t q = 0; q < n; ++q)
      if (hs[q] < 0 || hs[q] >= N || (h->flags[hs[q]] & 1))
        return fail(HHG_EINVAL, "slots must be non-Dirichlet slots of the mesh");
  }
  double *D = nullptr;
  HHG_HIP(hipMalloc((void **)&D, 6 * (size_t)N * sizeof(double)));
  rc = diag_blocks(h, k, method, D, st);
  if (!rc) {
    hipLaunchKernelGGL(k_collect, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h->d_minfo,
                       h->n_macro, k, r, e, D, N, slots, n, static_cast<uint16_t *>(samples));
    hipError_t le = hipGetLastError();
    if (le != hipSuccess) rc = hip_fail(le, "k_collect");
  }
  hipError_t se = hipStreamSynchronize(st);
  (void)hipFree(D);
  if (rc) return rc;
  if (se != hipSuccess) return hip_fail(se, "hipStreamSynchronize");
  return HHG_OK;
}

int hhg_mlp_loss_grad(hhg_mlp m, const void *samples, int64_t n, double *loss, float *grad,
                      void *stream) {
  int rc = check_model(m);
  if (rc) return rc;
  if (!samples || !loss || !grad) return fail(HHG_EINVAL, "null argument");
  if (n < 1) return fail(HHG_EINVAL, "n must be >= 1");
  if (!aligned(samples, 16)) return fail(HHG_EINVAL, "misaligned records");
  hipStream_t st = (hipStream_t)stream;
  TrainScratch ts;
  if ((rc = ts.alloc(n, 1))) return rc;
  float *dgrad = nullptr;
  HHG_HIP(hipMalloc((void **)&dgrad, NPARAM * sizeof(float)));
  rc = train_batch(m, static_cast<const uint16_t *>(samples), n, ts, ts.loss, dgrad, nullptr, st);
  if (!rc) {
    hipError_t e1 = hipMemcpyAsync(grad, dgrad, NPARAM * sizeof(float), hipMemcpyDeviceToHost, st);
    hipError_t e2 = hipMemcpyAsync(loss, ts.loss, sizeof(double), hipMemcpyDeviceToHost, st);
    hipError_t e3 = hipStreamSynchronize(st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
      rc = hip_fail(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3), "hhg_mlp_loss_grad");
  } else {
    (void)hipStreamSynchronize(st);
  }
  (void)hipFree(dgrad);
  return rc;
}

int hhg_mlp_train(hhg_mlp m, const void *samples, int64_t n, const hhg_train_opts *o,
                  float *loss_hist, void *stream) {
  int rc = check_model(m);
  if (rc) return rc;
  if (!samples || !o) return fail(HHG_EINVAL, "null argument");
  if (n < 1 || o->batch < 1 || o->epochs < 1) return fail(HHG_EINVAL, "n, batch and epochs must be >= 1");
  if (!(o->lr > 0.0f) || !(o->beta1 >= 0.0f && o->beta1 < 1.0f) ||
      !(o->beta2 >= 0.0f && o->beta2 < 1.0f) || !(o->eps >= 0.0f))
    return fail(HHG_EINVAL, "lr must be > 0, betas in [0, 1), eps >= 0");
  if (!aligned(samples, 16)) return fail(HHG_EINVAL, "misaligned records");
  hipStream_t st = (hipStream_t)stream;
  const int64_t B = std::min<int64_t>(o->batch, n);
  const int64_t per_epoch = (n + B - 1) / B;
  const int64_t steps = per_epoch * o->epochs;
  TrainScratch ts;
  if ((rc = ts.alloc(B, steps))) return rc;
  const uint16_t *rec = static_cast<const uint16_t *>(samples);
  for (int ep = 0; ep < o->epochs && !rc; ++ep)
    for (int64_t b = 0; b < per_epoch && !rc; ++b) {
      const int64_t a = b * B, len = std::min<int64_t>(B, n - a);
      rc = train_batch(m, rec + a * REC_U16, len, ts, ts.loss + ep * per_epoch + b, nullptr, o, st);
    }
  if (rc) {
    (void)hipStreamSynchronize(st);
    return rc;
  }
  std::vector<double> lb((size_t)steps);
  HHG_HIP(hipMemcpyAsync(lb.data(), ts.loss, steps * sizeof(double), hipMemcpyDeviceToHost, st));
  HHG_HIP(hipStreamSynchronize(st));
  if (loss_hist)
    for (int ep = 0; ep < o->epochs; ++ep) {
      double s = 0.0;
      for (int64_t b = 0; b < per_epoch; ++b) {
        const int64_t a = b * B, len = std::min<int64_t>(B, n - a);
        s += lb[ep * per_epoch + b] * (double)len;
      }
      loss_hist[ep] = (float)(s / (double)n);
    }
  return HHG_OK;
}

int hhg_set_learned_model(hhg_handle h, hhg_mlp m) {
  if (!h) return fail(HHG_EINVAL, "null handle");
  if (m) {
    int rc = check_model(m);
    if (rc) return rc;
  }
  h->model = m;
  return HHG_OK;
}

}  // extern "C"
