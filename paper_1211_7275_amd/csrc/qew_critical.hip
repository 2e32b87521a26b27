// qew_critical.hip -- critical force f_c^s and critical configuration u_c^s of
// samples periodic in u (Sec. III A of arXiv:1211.7275), on the device.
//
// The critical configuration is the pinned solution of
//   c d2u/dx2 + F_p(u, x) + f = 0                       (Sec. III A)
// with the largest f.  The Middleton theorems (no passing) make it reachable
// without integrating Eq. (1) in time:
//   - from a configuration whose forces are all >= 0, moving any site forward
//     to the first zero of its own force (neighbours held) keeps every force
//     >= 0 (the neighbours' forces only grow) and never passes a pinned
//     configuration that lies ahead (at a site of a pinned configuration ahead,
//     with neighbours behind theirs, the force is <= 0, so the first zero comes
//     no later).  Repeating such moves therefore climbs to the leftmost pinned
//     configuration ahead, if one exists;
//   - in a sample periodic in u the translates by M of a pinned configuration
//     are pinned too, so a line that advances by M everywhere has passed none:
//     there is no pinned configuration at that drive.
// Each workgroup owns one sample and runs a bisection on f: a trial drive is
// "pinned" when the forward moves converge (every |force| <= tol_force) and
// "depinned" when every site has advanced by M from the trial's start (the
// last pinned configuration), all in LDS within one launch.  The moves are
// applied to the even and then the odd sites (never two neighbours at once).
// The very first configuration (at the lower drive) is relaxed by moving each
// site to the nearest zero of its own force in the direction of the force,
// which lowers the line's energy at every move.
//
// Only the Catmull-Rom kinds (continuous forces) are handled; the local
// force of a site is a polynomial in its offset within a cell, and its first
// zero is found on the monotone pieces between the polynomial's turning
// points by Newton steps kept inside a shrinking bracket.
#include "qew_device.hpp"
#include "qew_internal.hpp"

namespace qew {

namespace {

// Threads of a workgroup: one per pair of sites, at most this many.
constexpr int kCritMaxBlock = 1024;
constexpr int kMaxCells = 64;        // cells one move may cross (then it stops at the cell edge)
constexpr int kBisect = 64;          // bound on the bracketed Newton steps of one zero
constexpr int kCheckEvery = 4;       // sweeps between convergence checks

// Local force of site j as a cubic in the offset s of cell n:
//   g(s) = A - 2c (n + s) + F_p(n + s),  A = c (u_{j-1} + u_{j+1}) + f.
struct Cubic {
  double b0, b1, b2, b3;
  __device__ double at(double s) const { return b0 + s * (b1 + s * (b2 + s * b3)); }
  __device__ double slope(double s) const { return b1 + s * (2.0 * b2 + s * (3.0 * b3)); }
};

constexpr double kEps = 2.220446049250313e-16;

// a / b (b != 0) to about an ulp: the hardware reciprocal refined by one
// Newton step.  The quotients below steer bracketed searches and place
// turning points, where an ulp more or less changes nothing, and the full
// IEEE division sequence is a long dependent chain on the critical path.
__device__ __forceinline__ double quot(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  return a * r;
}

// A point next to the zero of g on [lo, hi], where g is monotone with
// g(lo) = glo > 0 >= g(hi) = ghi (up) or glo >= 0 > ghi (down).  The answer
// lies on the near side of the zero -- g > 0 (up) or g < 0 (down) -- so a move
// there never passes it.  Newton steps are taken from the end with the
// smaller |g| and kept inside the bracket (a step that leaves it becomes the
// midpoint).  When that end is the far-side one and already within `tol` of
// zero, the next point is placed as far on the near side of the Newton
// estimate of the zero as the end lies on the other side, so that a function
// that keeps the Newton steps on the far side still yields a near-side point.
// Stops once the near-side end has |g| <= tol or the bracket is a few ulp
// wide.
__device__ double bracketed_zero(const Cubic& g, double lo, double hi, double glo, double ghi, bool up,
                                 double tol) {
  for (int it = 0; it < kBisect; ++it) {
    const double gn = up ? glo : ghi;
    if (fabs(gn) <= tol || hi - lo <= 4.0 * kEps) break;
    const bool from_lo = fabs(glo) <= fabs(ghi);
    const double e = from_lo ? lo : hi;
    const double ge = from_lo ? glo : ghi;
    const double d = g.slope(e);
    double x = (d != 0.0) ? e - quot(ge, d) : 0.5 * (lo + hi);
    if (from_lo != up && fabs(ge) <= tol) {
      const double off = fmax(fabs(e - x), 4.0 * kEps);
      x = up ? x - off : x + off;
    }
    if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
    const double gx = g.at(x);
    if (up ? (gx > 0.0) : (gx >= 0.0)) {
      lo = x;
      glo = gx;
    } else {
      hi = x;
      ghi = gx;
    }
  }
  return up ? lo : hi;
}

// The strength-scaled nodes n-1 .. n+2 of site j: the Catmull-Rom window of
// cell n.  The random-bond kind makes them one at a time: four FP64
// Box-Muller transforms at once would hold more registers than 1024 threads
// per workgroup leave (measured: the sequential form is faster there, the
// interleaved one for the uniform nodes).
template <int KIND>
__device__ void node_window(uint32_t j, int32_t n, uint32_t id, const CritParams& q, double p[4]) {
  if constexpr (KIND == kRF) {
#pragma unroll
    for (int i = 0; i < 4; ++i) p[i] = q.strength * node_f64<KIND>(j, n - 1 + i, id, q.k0, q.k1, q.period);
  } else {
#pragma unroll 1
    for (int i = 0; i < 4; ++i) p[i] = q.strength * node_f64<KIND>(j, n - 1 + i, id, q.k0, q.k1, q.period);
  }
}

// Local force in cell n from its window p.
template <int KIND>
__device__ Cubic cubic_of(const double p[4], int32_t n, double A, double c) {
  // Catmull-Rom in s: value = 1/2 [2 p1 + d1 s + d2 s^2 + d3 s^3]
  const double d1 = p[2] - p[0];
  const double d2 = 2.0 * p[0] - 5.0 * p[1] + 4.0 * p[2] - p[3];
  const double d3 = -p[0] + 3.0 * p[1] - 3.0 * p[2] + p[3];
  Cubic g;
  const double lin = A - 2.0 * c * (double)n;
  if constexpr (KIND == kRF) {  // F_p = value
    g.b0 = lin + p[1];
    g.b1 = -2.0 * c + 0.5 * d1;
    g.b2 = 0.5 * d2;
    g.b3 = 0.5 * d3;
  } else {  // random bond: F_p = -d value / ds
    g.b0 = lin - 0.5 * d1;
    g.b1 = -2.0 * c - d2;
    g.b2 = -1.5 * d3;
    g.b3 = 0.0;
  }
  return g;
}

// Turning points of g (roots of g') strictly inside (lo, hi), ascending; returns the count.
__device__ int turning_points(const Cubic& g, double lo, double hi, double t[2]) {
  const double a = 3.0 * g.b3, b = 2.0 * g.b2, c = g.b1;
  double r[2];
  int n = 0;
  if (a == 0.0) {
    if (b != 0.0) r[n++] = quot(-c, b);
  } else {
    const double disc = b * b - 4.0 * a * c;
    if (disc > 0.0) {
      const double q = -0.5 * (b + copysign(sqrt(disc), b));
      r[n++] = quot(q, a);
      if (q != 0.0) r[n++] = quot(c, q);
    } else if (disc == 0.0) {
      r[n++] = quot(-b, 2.0 * a);
    }
  }
  if (n == 2 && r[1] < r[0]) {
    const double x = r[0];
    r[0] = r[1];
    r[1] = x;
  }
  int m = 0;
  for (int i = 0; i < n; ++i)
    if (r[i] > lo && r[i] < hi) t[m++] = r[i];
  return m;
}

// First s in [s0, 1] where g (with g(s0) = g0 > 0) reaches 0, found on the
// monotone piece that holds the crossing; returns a point just short of it
// (g > 0 there, so a move never steps past the zero), or -1 if g > 0 on all
// of [s0, 1].
__device__ double first_zero_up(const Cubic& g, double s0, double g0, double tol) {
  double t[2];
  const int m = turning_points(g, s0, 1.0, t);
  double a = s0, ga = g0;
  for (int i = 0; i <= m; ++i) {
    const double b = (i < m) ? t[i] : 1.0;
    const double gb = g.at(b);
    if (gb <= 0.0) return bracketed_zero(g, a, b, ga, gb, true, tol);
    a = b;
    ga = gb;
  }
  return -1.0;
}

// Last s in [0, s0] where g (with g(s0) = g0 < 0) is 0 going down; returns a
// point just short of it (g < 0 there), or 2 if g < 0 on all of [0, s0].
__device__ double first_zero_down(const Cubic& g, double s0, double g0, double tol) {
  double t[2];
  const int m = turning_points(g, 0.0, s0, t);
  double b = s0, gb = g0;
  for (int i = m; i >= 0; --i) {
    const double a = (i > 0) ? t[i - 1] : 0.0;
    const double ga = g.at(a);
    if (ga >= 0.0) return bracketed_zero(g, a, b, ga, gb, false, tol);
    b = a;
    gb = ga;
  }
  return 2.0;
}

// Move of one site with its neighbours held: forward to the first zero of its
// force ahead (dir > 0) or backward to the first zero behind (dir < 0),
// starting at offset s of cell n with window p and local force g, g0 = g(s).
// A move into the next cell shifts the window by one node, so each cell
// crossed costs one node.  Returns the new position; the force left there is
// within `tol` of zero unless the bracket ran down to a few ulp first.
template <int KIND>
__device__ double relax_site(int32_t n, double s, double g0, Cubic g, double p[4], double A, uint32_t j,
                             uint32_t id, const CritParams& q, int dir, double tol) {
  for (int cell = 0; cell < kMaxCells; ++cell) {
    if (cell > 0) {
      g = cubic_of<KIND>(p, n, A, q.c);
      g0 = g.at(s);
    }
    if (dir > 0) {
      const double r = first_zero_up(g, s, g0, tol);
      if (r >= 0.0) return (double)n + r;
      n += 1;  // g > 0 across the rest of the cell: on to the next one
      s = 0.0;
      p[0] = p[1];
      p[1] = p[2];
      p[2] = p[3];
      p[3] = q.strength * node_f64<KIND>(j, n + 2, id, q.k0, q.k1, q.period);
    } else {
      const double r = first_zero_down(g, s, g0, tol);
      if (r <= 1.0) return (double)n + r;
      n -= 1;
      s = 1.0;
      p[3] = p[2];
      p[2] = p[1];
      p[1] = p[0];
      p[0] = q.strength * node_f64<KIND>(j, n - 1, id, q.k0, q.k1, q.period);
    }
  }
  return (double)n + s;  // a long move is continued in the next sweep
}

template <int KIND>
__device__ double force_at(double ul, double u, double ur, uint32_t j, uint32_t id, double f, const CritParams& q) {
  const double nf = floor(u);
  double p[4];
  node_window<KIND>(j, (int32_t)nf, id, q, p);
  const Cubic g = cubic_of<KIND>(p, (int32_t)nf, q.c * (ul + ur) + f, q.c);
  return g.at(u - nf);
}

// Block-wide max of a and min of b (every thread receives both).
__device__ void block_maxmin(double& a, double& b, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a = fmax(a, __shfl_xor(a, off, 64));
    b = fmin(b, __shfl_xor(b, off, 64));
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = a;
    red[2 * w + 1] = b;
  }
  __syncthreads();
  a = red[0];
  b = red[1];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
    a = fmax(a, red[2 * i]);
    b = fmin(b, red[2 * i + 1]);
  }
}

}  // namespace

// One workgroup per sample, one thread per pair of neighbouring sites (2t,
// 2t + 1), so every lane moves a site in both halves of a sweep.  LDS: u[L]
// (the trial), v[L] (the last pinned configuration, the trial's start),
// reduction scratch.
template <int KIND>
__global__ void __launch_bounds__(kCritMaxBlock)
    k_critical(CritParams q, const uint32_t* __restrict__ did, double* __restrict__ u_io,
               double* __restrict__ f_out, int64_t* __restrict__ st_out) {
  extern __shared__ double sh[];
  const int L = q.L;
  double* u = sh;
  double* v = sh + L;
  double* red = sh + 2 * L;
  const int s = blockIdx.x;
  const int nt = blockDim.x;
  const uint32_t id = did[s];
  for (int j = threadIdx.x; j < L; j += nt) u[j] = u_io[(int64_t)s * L + j];
  __syncthreads();

  int64_t sweeps = 0;
  int status = 0;
  // A site whose force is within tol_force / 4 of zero is left where it is,
  // and a move stops once the force left at the site is within tol_force / 64:
  // a converged line (every |force| <= tol_force) is reached without chasing
  // zeros to the last ulp.
  const double skip = 0.25 * q.tol_force;
  const double stop = q.tol_force * (1.0 / 64.0);
  // One sweep at drive f: the even sites, then the odd ones (the last site
  // alone when L is odd, since it neighbours site 0).  dir = +1: forward
  // moves; 0: towards the force.
  auto sweep = [&](double f, int dir) {
    const int npairs = L >> 1;  // sites 2t and 2t + 1 for t < npairs; an odd L's last site comes third
    const int phases = (L & 1) ? 3 : 2;
    for (int ph = 0; ph < phases; ++ph) {
      const int count = (ph < 2) ? npairs : 1;
      for (int t = threadIdx.x; t < count; t += nt) {
        const int j = (ph < 2) ? 2 * t + ph : L - 1;
        const double ul = u[j == 0 ? L - 1 : j - 1];
        const double ur = u[j == L - 1 ? 0 : j + 1];
        const double A = q.c * (ul + ur) + f;
        const double x = u[j];
        const double nf = floor(x);
        double p[4];
        node_window<KIND>((uint32_t)j, (int32_t)nf, id, q, p);
        const Cubic g = cubic_of<KIND>(p, (int32_t)nf, A, q.c);
        const double g0 = g.at(x - nf);
        int d = dir;
        if (d == 0) d = g0 > 0.0 ? 1 : (g0 < 0.0 ? -1 : 0);
        if ((d > 0 && g0 > skip) || (d < 0 && g0 < -skip))
          u[j] = relax_site<KIND>((int32_t)nf, x - nf, g0, g, p, A, (uint32_t)j, id, q, d, stop);
      }
      __syncthreads();
    }
  };
  // Largest |force| and smallest advance over the start v.
  auto check = [&](double f, double& fmax, double& adv) {
    fmax = 0.0;
    adv = INFINITY;
    for (int j = threadIdx.x; j < L; j += nt) {
      const double F = force_at<KIND>(u[j == 0 ? L - 1 : j - 1], u[j], u[j == L - 1 ? 0 : j + 1], (uint32_t)j,
                                      id, f, q);
      fmax = fmax > fabs(F) ? fmax : fabs(F);
      adv = fmin(adv, u[j] - v[j]);
    }
    block_maxmin(fmax, adv, red);
  };
  // Relax at drive f from the configuration in u; returns 0 pinned, 1
  // depinned (advanced by M over v everywhere), 2 undecided.
  auto relax = [&](double f, int dir) -> int {
    for (int64_t k = 0; k < q.max_sweeps; k += kCheckEvery) {
      for (int i = 0; i < kCheckEvery; ++i) sweep(f, dir);
      sweeps += kCheckEvery;
      double fmax, adv;
      check(f, fmax, adv);
      if (fmax <= q.tol_force) return 0;
      if (dir > 0 && adv >= (double)q.period) return 1;
    }
    return 2;
  };

  double f_lo = q.f_lo, f_hi = q.f_hi;
  for (int j = threadIdx.x; j < L; j += nt) v[j] = -INFINITY;  // no advance test at the lower drive
  __syncthreads();
  int r = relax(f_lo, 0);
  if (r != 0) {
    status = 1;  // no pinned configuration reached at the lower drive
  } else {
    for (int j = threadIdx.x; j < L; j += nt) v[j] = u[j];
    __syncthreads();
    for (int round = 0; round < q.max_rounds && f_hi - f_lo >= q.tol_f; ++round) {
      const double f_mid = 0.5 * (f_lo + f_hi);
      r = relax(f_mid, 1);
      if (r == 0) {
        f_lo = f_mid;
        for (int j = threadIdx.x; j < L; j += nt) v[j] = u[j];
      } else if (r == 1) {
        f_hi = f_mid;
        for (int j = threadIdx.x; j < L; j += nt) u[j] = v[j];
      } else {
        status = 2;  // a trial undecided within max_sweeps
        break;
      }
      __syncthreads();
    }
    if (status == 0 && f_hi - f_lo >= q.tol_f) status = 3;  // out of rounds
  }
  __syncthreads();
  for (int j = threadIdx.x; j < L; j += nt) u_io[(int64_t)s * L + j] = (status == 0) ? v[j] : u[j];
  if (threadIdx.x == 0) {
    f_out[2 * s] = f_lo;
    f_out[2 * s + 1] = f_hi;
    st_out[2 * s] = status;
    st_out[2 * s + 1] = sweeps;
  }
}

size_t critical_lds_bytes(int L) { return (size_t)(2 * L + 2 * (kCritMaxBlock / 64)) * sizeof(double); }

// Threads per workgroup: one per pair of sites, whole waves, at most kCritMaxBlock.
static int critical_block(int L) {
  const int pairs = L >> 1;
  const int t = ((pairs + 63) / 64) * 64;
  return t < 64 ? 64 : (t > kCritMaxBlock ? kCritMaxBlock : t);
}

hipError_t launch_critical(int kind, const CritParams& q, int n_samples, const uint32_t* did, double* u_io,
                           double* f_out, int64_t* st_out, hipStream_t st) {
  const size_t lds = critical_lds_bytes(q.L);
  const void* fn = kind == kRF ? reinterpret_cast<const void*>(&k_critical<kRF>)
                               : reinterpret_cast<const void*>(&k_critical<kRB>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (kind == kRF)
    hipLaunchKernelGGL(k_critical<kRF>, dim3(n_samples), dim3(critical_block(q.L)), lds, st, q, did, u_io, f_out, st_out);
  else
    hipLaunchKernelGGL(k_critical<kRB>, dim3(n_samples), dim3(critical_block(q.L)), lds, st, q, did, u_io, f_out, st_out);
  return hipGetLastError();
}

}  // namespace qew
