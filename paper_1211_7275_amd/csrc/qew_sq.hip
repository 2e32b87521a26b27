// qew_sq.hip -- structure factor S_q(t) of Eq. (6) of arXiv:1211.7275.
//
//   S_n = | L^-1 sum_x u_x exp(-i 2 pi n x / L) |^2,  q = 2 pi n / L,
//
// for every sample of a batch of equal power-of-two lengths L, in FP64, at a
// measurement step.  For real u the modes n and L - n are equal, so n = 1 ..
// L/2 is produced.  The real transform of length L is one complex transform
// of length N = L/2 on z_k = u_2k + i u_2k+1 (after subtracting the sample's
// first site, which only moves mode 0), followed by the usual split of the
// even and odd halves.  The complex transform is a Stockham auto-sort FFT in
// passes of radix 8, 64 and 8, 4 or 2: every pass reads and writes the batch
// once, coalesced, with twiddles from sincospi in FP64; the first pass packs z
// from the chain as it reads it.  The per-mode values are then
// averaged over the samples and over caller-given ranges of n (cut into
// chunks of modes), in a fixed order (no atomics), so repeated runs give
// identical bits.
#include "qew_internal.hpp"

namespace qew {

namespace {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// multiply by -i
__device__ __forceinline__ double2 mul_mi(double2 a) { return make_double2(a.y, -a.x); }

// In-register DFT of R points: X_q = sum_r v_r exp(-2 pi i r q / R).
template <int R>
__device__ __forceinline__ void dft(double2* v);

template <>
__device__ __forceinline__ void dft<2>(double2* v) {
  const double2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<4>(double2* v) {
  const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  const double2 s13 = cadd(v[1], v[3]), d13 = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(s02, s13);
  v[1] = cadd(d02, d13);
  v[2] = csub(s02, s13);
  v[3] = csub(d02, d13);
}

template <>
__device__ __forceinline__ void dft<8>(double2* v) {
  // radix-4 transforms of the even and odd points, then one radix-2 layer
  double2 e[4] = {v[0], v[2], v[4], v[6]};
  double2 o[4] = {v[1], v[3], v[5], v[7]};
  dft<4>(e);
  dft<4>(o);
  constexpr double h = 0.70710678118654752440;  // 1/sqrt(2)
  const double2 w1 = make_double2(h, -h), w3 = make_double2(-h, -h);
  const double2 t0 = o[0], t1 = cmul(o[1], w1), t2 = mul_mi(o[2]), t3 = cmul(o[3], w3);
  v[0] = cadd(e[0], t0);
  v[4] = csub(e[0], t0);
  v[1] = cadd(e[1], t1);
  v[5] = csub(e[1], t1);
  v[2] = cadd(e[2], t2);
  v[6] = csub(e[2], t2);
  v[3] = cadd(e[3], t3);
  v[7] = csub(e[3], t3);
}

// All transform lengths are powers of two, so every index split below is a
// shift or a mask.  blockIdx.y walks the samples (grid-stride for large S).

// Points of the complex transform: from the previous pass's buffer, or (the
// first pass) packed on the fly from the chain, z_m = (u_2m - K) + i (u_2m+1 - K)
// with K = u_0 of the sample.
enum { kSrcBuffer = 0, kSrcPlain = 1, kSrcSplit = 2 };
struct FftSource {
  const double2* buf;      // kSrcBuffer: [S][N]
  const int64_t* off;      // chains: sample offsets
  const double* u;         // kSrcPlain
  const int32_t* cell;     // kSrcSplit
  const float* frac;
};

template <int SRC>
__device__ __forceinline__ double sample_shift(const FftSource& src, int s) {
  if constexpr (SRC == kSrcPlain) return src.u[src.off[s]];
  else if constexpr (SRC == kSrcSplit) return (double)src.cell[src.off[s]] + (double)src.frac[src.off[s]];
  else return 0.0;
}

template <int SRC>
__device__ __forceinline__ double2 load_point(const FftSource& src, int s, int lgN, int m, double K) {
  if constexpr (SRC == kSrcBuffer) {
    return src.buf[((int64_t)s << lgN) + m];
  } else if constexpr (SRC == kSrcPlain) {
    const double2 x = *reinterpret_cast<const double2*>(src.u + src.off[s] + 2 * (int64_t)m);
    return make_double2(x.x - K, x.y - K);
  } else {
    const int64_t b = src.off[s] + 2 * (int64_t)m;
    const int2 c = *reinterpret_cast<const int2*>(src.cell + b);
    const float2 r = *reinterpret_cast<const float2*>(src.frac + b);
    return make_double2(((double)c.x + (double)r.x) - K, ((double)c.y + (double)r.y) - K);
  }
}

// One Stockham pass of radix R = 2^lgR over every transform of the batch:
// sub-transforms of Ns = 2^lgNs points are done, this pass makes them Ns * R.
// The twiddles exp(-2 pi i r k / (Ns R)) are powers of the r = 1 twiddle.
// The first pass of a transform (SRC = kSrcPlain or kSrcSplit) reads the
// chain itself; a wave then reads 64 consecutive points per load.
template <int R, int SRC>
__global__ void __launch_bounds__(kBlock)
    k_fft_pass(FftSource src, double2* __restrict__ out, int lgN, int lgNs, int S) {
  constexpr int lgR = R == 8 ? 3 : (R == 4 ? 2 : 1);
  const int NR = 1 << (lgN - lgR);
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= NR) return;
  const int k = j & ((1 << lgNs) - 1);
  const int base = ((j >> lgNs) << (lgNs + lgR)) + k;
  double2 w1 = make_double2(1.0, 0.0);
  if (lgNs > 0) {
    double sn, cs;
    sincospi(-2.0 * (double)k / (double)(1 << (lgNs + lgR)), &sn, &cs);
    w1 = make_double2(cs, sn);
  }
  for (int s = blockIdx.y; s < S; s += gridDim.y) {
    const double K = sample_shift<SRC>(src, s);
    double2* o = out + ((int64_t)s << lgN);
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = load_point<SRC>(src, s, lgN, j + r * NR, K);
    if (lgNs > 0) {
      double2 w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        v[r] = cmul(v[r], w);
        w = cmul(w, w1);
      }
    }
    dft<R>(v);
#pragma unroll
    for (int q = 0; q < R; ++q) o[base + (q << lgNs)] = v[q];
  }
}

// One Stockham pass of radix 64 = 8 x 8 over every transform of the batch,
// the same indexing as k_fft_pass with R = 64, so it reads and writes the
// batch once where three radix-8 passes would do it three times.  A wave
// covers 8 consecutive j (jj = lane & 7) with 8 threads each (t = lane >> 3):
// thread t loads the points r = t + 8 r2 (r2 = 0..7), twiddles them, and
// transforms over r2; after the inner twiddle exp(-2 pi i t q2 / 64) the
// wave exchanges the 8 x 8 block of each j through LDS, thread t takes q2 = t
// and transforms over r1, giving the outputs q = t + 8 q1.  Every load and
// store instruction of a wave moves 8 runs of 8 consecutive points (128 B).
// The exchange stays inside the wave, whose LDS operations complete in order,
// so no workgroup barrier is needed.
__global__ void __launch_bounds__(kBlock)
    k_fft_pass64(const double2* __restrict__ in, double2* __restrict__ out, int lgN, int lgNs, int S) {
  constexpr int kPad = 9;  // row stride of the exchange block (against bank conflicts)
  __shared__ double2 xch[kBlock / 64][8][8 * kPad];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int jj = lane & 7, t = lane >> 3;
  const int NR = 1 << (lgN - 6);
  const int j = (blockIdx.x * (kBlock / 64) + wv) * 8 + jj;
  const bool active = j < NR;
  const int k = j & ((1 << lgNs) - 1);
  // Twiddles (independent of the sample): the pass's exp(-2 pi i r k / (64 Ns))
  // for r = t + 8 r2 as a b^r2 with a = exp(-2 pi i t k / (64 Ns)) and
  // b = exp(-2 pi i 8 k / (64 Ns)), and the inner exp(-2 pi i t q2 / 64) as c^q2.
  double2 tw[8], iw[8];
  {
    double sn, cs;
    sincospi(-2.0 * (double)(t * (int64_t)k) / (double)(64 << lgNs), &sn, &cs);
    const double2 a = make_double2(cs, sn);
    sincospi(-2.0 * (double)(8 * (int64_t)k) / (double)(64 << lgNs), &sn, &cs);
    const double2 b = make_double2(cs, sn);
    sincospi(-2.0 * (double)t / 64.0, &sn, &cs);
    const double2 c = make_double2(cs, sn);
    tw[0] = a;
    iw[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int i = 1; i < 8; ++i) {
      tw[i] = cmul(tw[i - 1], b);
      iw[i] = cmul(iw[i - 1], c);
    }
  }
  const int base = ((j >> lgNs) << (lgNs + 6)) + k;
  double2* row = &xch[wv][jj][0];
  for (int s = blockIdx.y; s < S; s += gridDim.y) {
    const double2* a = in + ((int64_t)s << lgN);
    double2* o = out + ((int64_t)s << lgN);
    double2 v[8];
#pragma unroll
    for (int r2 = 0; r2 < 8; ++r2) v[r2] = active ? a[j + (t + 8 * r2) * NR] : make_double2(0.0, 0.0);
    if (lgNs > 0) {
#pragma unroll
      for (int r2 = 0; r2 < 8; ++r2) v[r2] = cmul(v[r2], tw[r2]);
    }
    dft<8>(v);  // over r2: v[q2]
#pragma unroll
    for (int q2 = 1; q2 < 8; ++q2) v[q2] = cmul(v[q2], iw[q2]);
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) row[t * kPad + q2] = v[q2];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r1 = 0; r1 < 8; ++r1) v[r1] = row[r1 * kPad + t];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    dft<8>(v);  // over r1: v[q1] = output t + 8 q1
    if (active) {
#pragma unroll
      for (int q1 = 0; q1 < 8; ++q1) o[base + ((t + 8 * q1) << lgNs)] = v[q1];
    }
  }
}

// Real transform from the half-length complex one, and S_n = |U_n / L|^2 for
// n = 0 .. N (sq[s][n], row length N + 1).
__global__ void __launch_bounds__(kBlock)
    k_sq_post(const double2* __restrict__ Z, double* __restrict__ sq, int N, int S, double inv_l2) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n > N) return;
  double sn, cs;
  sincospi(-(double)n / (double)N, &sn, &cs);  // exp(-2 pi i n / L)
  const double2 W = make_double2(cs, sn);
  for (int s = blockIdx.y; s < S; s += gridDim.y) {
    const double2* zs = Z + (int64_t)s * N;
    const double2 zn = zs[n == N ? 0 : n];
    const double2 zc = zs[n == 0 ? 0 : N - n];
    const double2 zm = make_double2(zc.x, -zc.y);  // conj(Z_{N-n})
    const double2 A = make_double2(0.5 * (zn.x + zm.x), 0.5 * (zn.y + zm.y));
    const double2 D = csub(zn, zm);
    const double2 B = make_double2(0.5 * D.y, -0.5 * D.x);  // D / (2i)
    const double2 U = cadd(A, cmul(W, B));
    sq[(int64_t)s * (N + 1) + n] = (U.x * U.x + U.y * U.y) * inv_l2;
  }
}

// Mean over the samples of every mode (samples in order).
__global__ void __launch_bounds__(kBlock)
    k_sq_mean(const double* __restrict__ sq, double* __restrict__ mean, int N, int S) {
  const int n = blockIdx.x * kBlock + threadIdx.x;
  if (n > N) return;
  double acc = 0.0;
  for (int s = 0; s < S; ++s) acc += sq[(int64_t)s * (N + 1) + n];
  mean[n] = acc / (double)S;
}

// Chunk c: sum of mean[n] over its modes (fixed order: thread stride, then a
// tree).
__global__ void __launch_bounds__(kBlock)
    k_sq_chunk(const double* __restrict__ mean, const int32_t* __restrict__ chunk_lo, double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int c = blockIdx.x;
  const int lo = chunk_lo[c], hi = chunk_lo[c + 1];
  double acc = 0.0;
  for (int n = lo + threadIdx.x; n < hi; n += kBlock) acc += mean[n];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c] = red[0];
}

// Bin b: its chunks' sums in order, divided by its number of modes.
__global__ void __launch_bounds__(kBlock)
    k_sq_bin(const double* __restrict__ part, const int32_t* __restrict__ chunk_lo,
             const int32_t* __restrict__ chunk_first, int n_bins, double* __restrict__ out) {
  const int b = blockIdx.x * kBlock + threadIdx.x;
  if (b >= n_bins) return;
  const int c0 = chunk_first[b], c1 = chunk_first[b + 1];
  double acc = 0.0;
  for (int c = c0; c < c1; ++c) acc += part[c];
  out[b] = acc / (double)(chunk_lo[c1] - chunk_lo[c0]);
}

dim3 grid2(int64_t n, int S) {
  const unsigned gx = (unsigned)((n + kBlock - 1) / kBlock);
  return dim3(gx < 1 ? 1 : gx, (unsigned)(S < 65535 ? S : 65535));
}

}  // namespace

hipError_t launch_sq(const int64_t* off, int S, int64_t L, const double* u_plain, SplitBuf split,
                     double2* bufA, double2* bufB, const int32_t* chunk_lo, int n_chunks,
                     const int32_t* chunk_first, int n_bins, double* part, double* out,
                     hipStream_t st) {
  const int N = (int)(L / 2);
  int lgN = 0;
  while ((1 << lgN) < N) ++lgN;
  hipError_t e = hipSuccess;
  double2* in = bufA;
  double2* outb = bufB;
  // The first pass (radix 8, or 4 for L = 8: the plan admits L >= 8) packs the
  // chain as it reads it; radix-64 passes follow while 64 or more points per
  // sub-transform remain to be combined, then radix 8, 4 or 2.
  const FftSource chain{nullptr, off, u_plain, split.cell, split.frac};
  const int lg0 = lgN >= 3 ? 3 : 2;
  {
    const dim3 g = grid2(N >> lg0, S);
    if (u_plain) {
      if (lg0 == 3) hipLaunchKernelGGL((k_fft_pass<8, kSrcPlain>), g, dim3(kBlock), 0, st, chain, in, lgN, 0, S);
      else hipLaunchKernelGGL((k_fft_pass<4, kSrcPlain>), g, dim3(kBlock), 0, st, chain, in, lgN, 0, S);
    } else {
      if (lg0 == 3) hipLaunchKernelGGL((k_fft_pass<8, kSrcSplit>), g, dim3(kBlock), 0, st, chain, in, lgN, 0, S);
      else hipLaunchKernelGGL((k_fft_pass<4, kSrcSplit>), g, dim3(kBlock), 0, st, chain, in, lgN, 0, S);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  int lgNs = lg0;
  while (lgNs < lgN) {
    const int rem = lgN - lgNs;
    const int lgR = rem >= 6 ? 6 : (rem >= 3 ? 3 : rem);
    const dim3 g = grid2(N >> lgR, S);
    const FftSource buf{in, nullptr, nullptr, nullptr, nullptr};
    if (lgR == 6)
      hipLaunchKernelGGL(k_fft_pass64, grid2((int64_t)(N >> 6) * 8, S), dim3(kBlock), 0, st, in, outb, lgN, lgNs, S);
    else if (lgR == 3)
      hipLaunchKernelGGL((k_fft_pass<8, kSrcBuffer>), g, dim3(kBlock), 0, st, buf, outb, lgN, lgNs, S);
    else if (lgR == 2)
      hipLaunchKernelGGL((k_fft_pass<4, kSrcBuffer>), g, dim3(kBlock), 0, st, buf, outb, lgN, lgNs, S);
    else
      hipLaunchKernelGGL((k_fft_pass<2, kSrcBuffer>), g, dim3(kBlock), 0, st, buf, outb, lgN, lgNs, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    lgNs += lgR;
    double2* t = in;
    in = outb;
    outb = t;
  }
  // `in` holds the transform; the other buffer takes S rows of N + 1 doubles
  // and, after them, the per-mode mean over the samples.
  double* sq = reinterpret_cast<double*>(outb);
  double* mean = sq + (int64_t)S * (N + 1);
  hipLaunchKernelGGL(k_sq_post, grid2(N + 1, S), dim3(kBlock), 0, st, in, sq, N, S,
                     1.0 / ((double)L * (double)L));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sq_mean, grid2(N + 1, 1), dim3(kBlock), 0, st, sq, mean, N, S);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sq_chunk, dim3(n_chunks), dim3(kBlock), 0, st, mean, chunk_lo, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sq_bin, dim3((n_bins + kBlock - 1) / kBlock), dim3(kBlock), 0, st, part, chunk_lo,
                     chunk_first, n_bins, out);
  return hipGetLastError();
}

}  // namespace qew
