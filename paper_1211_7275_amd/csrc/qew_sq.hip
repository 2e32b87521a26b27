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
// passes of radix 8 (then 4 or 2): every pass reads and writes the batch once,
// coalesced, with twiddles from sincospi in FP64.  The per-mode values are then
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

// z[s][k] = (u_2k - K) + i (u_2k+1 - K), K = u_0 of sample s.
__global__ void __launch_bounds__(kBlock)
    k_sq_pack_plain(const int64_t* __restrict__ off, const double* __restrict__ u, double2* __restrict__ z,
                    int N, int S) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= N) return;
  for (int s = blockIdx.y; s < S; s += gridDim.y) {
    const double* us = u + off[s];
    const double K = us[0];
    z[(int64_t)s * N + k] = make_double2(us[2 * k] - K, us[2 * k + 1] - K);
  }
}

__global__ void __launch_bounds__(kBlock)
    k_sq_pack_split(const int64_t* __restrict__ off, const int32_t* __restrict__ cell,
                    const float* __restrict__ frac, double2* __restrict__ z, int N, int S) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= N) return;
  for (int s = blockIdx.y; s < S; s += gridDim.y) {
    const int64_t b = off[s];
    const double K = (double)cell[b] + (double)frac[b];
    const double a0 = (double)cell[b + 2 * k] + (double)frac[b + 2 * k];
    const double a1 = (double)cell[b + 2 * k + 1] + (double)frac[b + 2 * k + 1];
    z[(int64_t)s * N + k] = make_double2(a0 - K, a1 - K);
  }
}

// One Stockham pass of radix R = 2^lgR over every transform of the batch:
// sub-transforms of Ns = 2^lgNs points are done, this pass makes them Ns * R.
// The twiddles exp(-2 pi i r k / (Ns R)) are powers of the r = 1 twiddle.
template <int R>
__global__ void __launch_bounds__(kBlock)
    k_fft_pass(const double2* __restrict__ in, double2* __restrict__ out, int lgN, int lgNs, int S) {
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
    const double2* a = in + ((int64_t)s << lgN);
    double2* o = out + ((int64_t)s << lgN);
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[j + r * NR];
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
  if (u_plain)
    hipLaunchKernelGGL(k_sq_pack_plain, grid2(N, S), dim3(kBlock), 0, st, off, u_plain, bufA, N, S);
  else
    hipLaunchKernelGGL(k_sq_pack_split, grid2(N, S), dim3(kBlock), 0, st, off, split.cell, split.frac,
                       bufA, N, S);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double2* in = bufA;
  double2* outb = bufB;
  for (int lgNs = 0; lgNs < lgN;) {
    const int rem = lgN - lgNs;
    const int lgR = rem >= 3 ? 3 : rem;
    const dim3 g = grid2(N >> lgR, S);
    if (lgR == 3)
      hipLaunchKernelGGL((k_fft_pass<8>), g, dim3(kBlock), 0, st, in, outb, lgN, lgNs, S);
    else if (lgR == 2)
      hipLaunchKernelGGL((k_fft_pass<4>), g, dim3(kBlock), 0, st, in, outb, lgN, lgNs, S);
    else
      hipLaunchKernelGGL((k_fft_pass<2>), g, dim3(kBlock), 0, st, in, outb, lgN, lgNs, S);
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
