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
// averaged over the samples and over caller-given ranges of n, in a fixed
// order (no atomics), so repeated runs give identical bits.
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

// z[s][k] = (u_2k - K) + i (u_2k+1 - K), K = u_0 of sample s.
__global__ void __launch_bounds__(kBlock)
    k_sq_pack_plain(const int64_t* __restrict__ off, const double* __restrict__ u, double2* __restrict__ z,
                    int64_t N, int64_t total) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t s = i / N, k = i - s * N;
    const double* us = u + off[s];
    const double K = us[0];
    z[i] = make_double2(us[2 * k] - K, us[2 * k + 1] - K);
  }
}

__global__ void __launch_bounds__(kBlock)
    k_sq_pack_split(const int64_t* __restrict__ off, const int32_t* __restrict__ cell,
                    const float* __restrict__ frac, double2* __restrict__ z, int64_t N, int64_t total) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t s = i / N, k = i - s * N;
    const int64_t b = off[s];
    const double K = (double)cell[b] + (double)frac[b];
    const double a0 = (double)cell[b + 2 * k] + (double)frac[b + 2 * k];
    const double a1 = (double)cell[b + 2 * k + 1] + (double)frac[b + 2 * k + 1];
    z[i] = make_double2(a0 - K, a1 - K);
  }
}

// One Stockham pass of radix R over every transform of the batch: Ns points of
// each sub-transform are done, this pass makes them Ns * R.
template <int R>
__global__ void __launch_bounds__(kBlock)
    k_fft_pass(const double2* __restrict__ in, double2* __restrict__ out, int64_t N, int64_t Ns,
               int64_t total) {
  const int64_t NR = N / R;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t s = i / NR, j = i - s * NR;
    const double2* a = in + s * N;
    double2* o = out + s * N;
    const int64_t k = j % Ns;
    double2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = a[j + r * NR];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double sn, cs;
        sincospi(-2.0 * (double)(r * k) / (double)(Ns * R), &sn, &cs);
        v[r] = cmul(v[r], make_double2(cs, sn));
      }
    }
    dft<R>(v);
    const int64_t base = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) o[base + q * Ns] = v[q];
  }
}

// Real transform from the half-length complex one, and S_n = |U_n / L|^2 for
// n = 0 .. N (sq[s][n], row length N + 1).
__global__ void __launch_bounds__(kBlock)
    k_sq_post(const double2* __restrict__ Z, double* __restrict__ sq, int64_t N, int64_t total,
              double inv_l2) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
    const int64_t s = i / (N + 1), n = i - s * (N + 1);
    const double2* zs = Z + s * N;
    const double2 zn = zs[n == N ? 0 : n];
    const double2 zc = zs[n == 0 ? 0 : N - n];
    const double2 zm = make_double2(zc.x, -zc.y);  // conj(Z_{N-n})
    const double2 A = make_double2(0.5 * (zn.x + zm.x), 0.5 * (zn.y + zm.y));
    const double2 D = csub(zn, zm);
    const double2 B = make_double2(0.5 * D.y, -0.5 * D.x);  // D / (2i)
    double sn, cs;
    sincospi(-(double)n / (double)N, &sn, &cs);  // exp(-2 pi i n / L)
    const double2 U = cadd(A, cmul(make_double2(cs, sn), B));
    sq[i] = (U.x * U.x + U.y * U.y) * inv_l2;
  }
}

// Bin b: mean of sq[s][n] over every sample s and n in [edges[b], edges[b+1]).
__global__ void __launch_bounds__(kBlock)
    k_sq_bin(const double* __restrict__ sq, int64_t N, int S, const int64_t* __restrict__ edges,
             double* __restrict__ out) {
  __shared__ double red[kBlock];
  const int b = blockIdx.x;
  const int64_t lo = edges[b], w = edges[b + 1] - lo;
  const int64_t total = (int64_t)S * w;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < total; e += kBlock) {
    const int64_t s = e / w;
    acc += sq[s * (N + 1) + lo + (e - s * w)];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0] / (double)total;
}

int grid_for(int64_t total) {
  const int64_t g = (total + kBlock - 1) / kBlock;
  return (int)(g < 65536 ? (g < 1 ? 1 : g) : 65536);
}

}  // namespace

hipError_t launch_sq(const int64_t* off, int S, int64_t L, const double* u_plain, SplitBuf split,
                     double2* bufA, double2* bufB, const int64_t* edges, int n_bins, double* out,
                     hipStream_t st) {
  const int64_t N = L / 2;
  int64_t total = (int64_t)S * N;
  if (u_plain)
    hipLaunchKernelGGL(k_sq_pack_plain, dim3(grid_for(total)), dim3(kBlock), 0, st, off, u_plain, bufA, N, total);
  else
    hipLaunchKernelGGL(k_sq_pack_split, dim3(grid_for(total)), dim3(kBlock), 0, st, off, split.cell, split.frac,
                       bufA, N, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double2* in = bufA;
  double2* outb = bufB;
  for (int64_t Ns = 1; Ns < N;) {
    const int64_t rem = N / Ns;
    const int R = rem >= 8 ? 8 : (int)rem;
    const int64_t work = (int64_t)S * (N / R);
    if (R == 8)
      hipLaunchKernelGGL((k_fft_pass<8>), dim3(grid_for(work)), dim3(kBlock), 0, st, in, outb, N, Ns, work);
    else if (R == 4)
      hipLaunchKernelGGL((k_fft_pass<4>), dim3(grid_for(work)), dim3(kBlock), 0, st, in, outb, N, Ns, work);
    else
      hipLaunchKernelGGL((k_fft_pass<2>), dim3(grid_for(work)), dim3(kBlock), 0, st, in, outb, N, Ns, work);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    Ns *= R;
    double2* t = in;
    in = outb;
    outb = t;
  }
  // `in` holds the transform; the other buffer takes S rows of N + 1 doubles.
  double* sq = reinterpret_cast<double*>(outb);
  total = (int64_t)S * (N + 1);
  hipLaunchKernelGGL(k_sq_post, dim3(grid_for(total)), dim3(kBlock), 0, st, in, sq, N, total,
                     1.0 / ((double)L * (double)L));
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sq_bin, dim3(n_bins), dim3(kBlock), 0, st, sq, N, S, edges, out);
  return hipGetLastError();
}

}  // namespace qew
