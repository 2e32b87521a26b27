// qew_kernels.hip -- gfx950 kernels of the QEW integrator.
//
// Eq. (1) of arXiv:1211.7275 (eta = 1) on periodic chains, explicit Euler
// (Sec. III B), pinning force from counter-based random values at integer u
// with a Catmull-Rom spline, and the FP64 observables of Eqs. (3)-(5).
//
// Kernels:
//   k_step_plain   one FP64 Euler step per launch, one thread per site, four
//                  Philox nodes regenerated per site update.  HBM traffic is
//                  16 B per update (read u, write u; neighbours hit L1/L2).
//   k_step_split1  the same on the split state (int32 cell + FP32 offset).
//   k_step_fused   `nsub` split Euler steps per launch.  Each workgroup owns
//                  a tile of 256*P consecutive sites held in registers (P
//                  per thread), `halo` of them on each side recomputed
//                  redundantly; the four nodes of each site's cell stay in
//                  LDS (and in HBM between launches).  A site whose cell
//                  changes needs one new node; each wave gathers its sites'
//                  requests into LDS and serves them with its own lanes, so
//                  Philox costs one pass per wave and sub-step instead of
//                  one per changed site slot.
//   k_meas_*       per-tile FP64 partials of sum F, sum (u-K), sum (u-K)^2.
//   k_meas_final   per-sample combine (Chan et al. pairwise update) into
//                  v, ubar, w2.
#include "qew_device.hpp"
#include "qew_internal.hpp"

namespace qew {

namespace {

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Wave-wide lane shifts by one (DPP wave_shr:1 / wave_shl:1): lane l receives
// x of lane l - 1 (resp. l + 1); lane 0 (resp. 63) receives 0.
__device__ __forceinline__ float from_lower_lane(float x) {
  const int v = __float_as_int(x);
  return __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_upper_lane(float x) {
  const int v = __float_as_int(x);
  return __int_as_float(__builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true));
}

// A pointer into LDS (32-bit, address space 3).
typedef __attribute__((address_space(3))) float lds_f32;

__device__ __forceinline__ uint32_t mbcnt64(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Block-wide deterministic FP64 sum of three values (fixed reduction order).
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double* lds /*[3*4]*/) {
  a = wave_sum_f64(a);
  b = wave_sum_f64(b);
  c = wave_sum_f64(c);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    lds[w * 3 + 0] = a;
    lds[w * 3 + 1] = b;
    lds[w * 3 + 2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0, z = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) {
      x += lds[i * 3 + 0];
      y += lds[i * 3 + 1];
      z += lds[i * 3 + 2];
    }
    a = x;
    b = y;
    c = z;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Initialisation: flat start u = 0 (Sec. II).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_init_plain(Tables t, double* u) {
  const int tile = blockIdx.x;
  const int s = t.mt_s[tile];
  const int p0 = t.mt_p0[tile], len = t.mt_len[tile];
  const int64_t base = t.off[s];
  for (int q = threadIdx.x; q < len; q += kBlock) u[base + p0 + q] = 0.0;
}

template <int KIND>
__global__ void __launch_bounds__(kBlock)
    k_init_split(Tables t, SplitBuf b, Phys ph, int with_nodes) {
  const int tile = blockIdx.x;
  const int s = t.mt_s[tile];
  const int p0 = t.mt_p0[tile], len = t.mt_len[tile];
  const int64_t base = t.off[s];
  const uint32_t id = t.did[s];
  const VectorKeys keys = vector_keys(ph.k0, ph.k1);
  for (int q = threadIdx.x; q < len; q += kBlock) {
    const int j = p0 + q;
    const int32_t c = 0;
    b.cell[base + j] = 0;
    b.frac[base + j] = 0.0f;
    if (with_nodes) {
      float4 nd;
      nd.x = node_f32<KIND>(j, c - 1, id, keys, ph.period);
      nd.y = node_f32<KIND>(j, c, id, keys, ph.period);
      nd.z = node_f32<KIND>(j, c + 1, id, keys, ph.period);
      nd.w = node_f32<KIND>(j, c + 2, id, keys, ph.period);
      b.nodes[base + j] = nd;
    }
  }
}

// Rebuild of the fused path's node cache for the state in `b` (after
// one-step stretches or a written state): the nodes of every site's cell.
template <int KIND>
__global__ void __launch_bounds__(kBlock) k_refresh_nodes(Tables t, SplitBuf b, Phys ph) {
  const int tile = blockIdx.x;
  const int s = t.mt_s[tile];
  const int p0 = t.mt_p0[tile], len = t.mt_len[tile];
  const int64_t base = t.off[s];
  const uint32_t id = t.did[s];
  const VectorKeys keys = vector_keys(ph.k0, ph.k1);
  for (int q = threadIdx.x; q < len; q += kBlock) {
    const int j = p0 + q;
    const int32_t c = b.cell[base + j];
    float4 nd;
    nd.x = node_f32<KIND>(j, c - 1, id, keys, ph.period);
    nd.y = node_f32<KIND>(j, c, id, keys, ph.period);
    nd.z = node_f32<KIND>(j, c + 1, id, keys, ph.period);
    nd.w = node_f32<KIND>(j, c + 2, id, keys, ph.period);
    b.nodes[base + j] = nd;
  }
}

// ---------------------------------------------------------------------------
// One-step kernels (one Euler step per launch).
// ---------------------------------------------------------------------------
// MEAS: also write the measurement partial of the input state (the same
// loop, forces and reduction order as k_meas_plain, so the partials are the
// same bits), so a measured step reads the state once.
template <int KIND, bool MEAS>
__global__ void __launch_bounds__(kBlock)
    k_step_plain(Tables t, const double* __restrict__ uin, double* __restrict__ uout, Phys ph,
                 Partial* part) {
  __shared__ double lds[MEAS ? 3 * (kBlock / 64) : 1];
  const int tile = blockIdx.x;
  const int s = t.mt_s[tile];
  const int p0 = t.mt_p0[tile], len = t.mt_len[tile];
  const int L = t.L[s];
  const int64_t base = t.off[s];
  const uint32_t id = t.did[s];
  const double f = t.f[s];
  const PlainPhys pp{ph.c, ph.dt, ph.strength};
  const VectorKeys keys = vector_keys(ph.k0, ph.k1);
  const double K = MEAS ? uin[base + p0] : 0.0;
  double sf = 0.0, s1 = 0.0, s2 = 0.0;
  for (int q = threadIdx.x; q < len; q += kBlock) {
    const int j = p0 + q;
    const int jm = (j == 0) ? L - 1 : j - 1;
    const int jp = (j == L - 1) ? 0 : j + 1;
    const double u = uin[base + j];
    const double F = plain_force<KIND>(uin[base + jm], u, uin[base + jp], (uint32_t)j, id, keys, f,
                                       ph.period, pp);
    uout[base + j] = u + ph.dt * F;
    if constexpr (MEAS) {
      sf += F;
      const double x = u - K;
      s1 += x;
      s2 += x * x;
    }
  }
  if constexpr (MEAS) {
    block_sum3(sf, s1, s2, lds);
    if (threadIdx.x == 0) part[tile] = Partial{sf, s1, s2, K};
  }
}

template <int KIND>
__device__ __forceinline__ void nodes_of(uint32_t j, int32_t c, uint32_t id, const Phys& ph,
                                         const VectorKeys& keys, float& p0, float& p1, float& p2,
                                         float& p3) {
  if (ph.strength == 0.0) {
    p0 = p1 = p2 = p3 = 0.0f;
    return;
  }
  // Catmull-Rom needs nodes c-1..c+2, Case 3 c..c+1, Case 4 c only.
  constexpr bool cubic = (KIND == kRF || KIND == kRB);
  p0 = cubic ? node_f32<KIND>(j, c - 1, id, keys, ph.period) : 0.0f;
  p1 = node_f32<KIND>(j, c, id, keys, ph.period);
  p2 = (KIND != kRFPc) ? node_f32<KIND>(j, c + 1, id, keys, ph.period) : 0.0f;
  p3 = cubic ? node_f32<KIND>(j, c + 2, id, keys, ph.period) : 0.0f;
}

// MEAS: also write the measurement partial of the input state, as
// k_meas_split computes it (same loop, forces and reduction order).
template <int KIND, bool MEAS>
__global__ void __launch_bounds__(kBlock)
    k_step_split1(Tables t, SplitBuf in, SplitBuf out, Phys ph, Partial* part) {
  __shared__ double lds[MEAS ? 3 * (kBlock / 64) : 1];
  const int tile = blockIdx.x;
  const int s = t.mt_s[tile];
  const int p0 = t.mt_p0[tile], len = t.mt_len[tile];
  const int L = t.L[s];
  const int64_t base = t.off[s];
  const uint32_t id = t.did[s];
  const float f = t.f32[s];
  const SplitPhys sp{ph.cf, ph.dtf, ph.sgn_strf};
  const int32_t Kc = MEAS ? in.cell[base + p0] : 0;
  const double Kr = MEAS ? (double)in.frac[base + p0] : 0.0;
  const VectorKeys keys = vector_keys(ph.k0, ph.k1);
  double sf = 0.0, s1 = 0.0, s2 = 0.0;
  for (int q = threadIdx.x; q < len; q += kBlock) {
    const int j = p0 + q;
    const int jm = (j == 0) ? L - 1 : j - 1;
    const int jp = (j == L - 1) ? 0 : j + 1;
    int32_t c = in.cell[base + j];
    float r = in.frac[base + j];
    float n0, n1, n2, n3;
    nodes_of<KIND>((uint32_t)j, c, id, ph, keys, n0, n1, n2, n3);
    const float4 a = spline_coef<KIND>(n0, n1, n2, n3, sp.sgn_str, f);
    const float F = split_force<KIND>(c, r, in.cell[base + jm], in.frac[base + jm],
                                      in.cell[base + jp], in.frac[base + jp], a, sp.c);
    if constexpr (MEAS) {
      sf += (double)F;
      const double x = (double)(c - Kc) + ((double)r - Kr);  // exact
      s1 += x;
      s2 += x * x;
    }
    c += (int32_t)split_advance(r, F, sp.dt);
    out.cell[base + j] = c;
    out.frac[base + j] = r;
  }
  if constexpr (MEAS) {
    block_sum3(sf, s1, s2, lds);
    if (threadIdx.x == 0) part[tile] = Partial{sf, s1, s2, (double)Kc + Kr};
  }
}

// ---------------------------------------------------------------------------
// Fused temporally blocked kernel (split precision).
//
// One workgroup owns one tile of T = 256 P consecutive sites of one sample at
// a time: positions p0 - halo .. p0 - halo + T - 1 (periodic in the sample).
// Thread t holds sites t P .. t P + P - 1 in registers: the cell as an exact
// float relative to the tile's first cell (no int/float conversion per step),
// the offset, and the coefficients of f + F_p of the current cell.  The four
// raw nodes of every site live in LDS, slot-major (node index i * 256 + t).
// Each sub-step:
//   1. every site takes one Euler step (neighbours within a thread directly,
//      across lanes by DPP wave shifts, across waves through a double-buffered
//      LDS edge array);
//   2. a site whose cell changed posts a request (its LDS node index and its
//      new and old cells) into its wave's region of the request list;
//   3. the same wave serves its requests, lane q taking request q: shift the
//      node window, generate the missing node (all four after a jump of two
//      or more cells), store the window, and write the new coefficients into
//      the request slot; the requesters then read them back.  Requests,
//      windows and replies belong to one wave and a wave's LDS operations
//      complete in order, so this needs no workgroup barrier;
//   4. the wave publishes its end sites; one workgroup barrier.
// A wave posts at most kReqPerWave requests per sub-step; the lanes of further
// requests (a burst of simultaneous cell changes) regenerate their windows
// themselves.  After nsub <= halo sub-steps the sites within `halo` of either
// tile end hold garbage (the tile ends reflect), and the valid part
// [halo, halo + len) is written back with its nodes.  Every value equals what
// the one-step kernel computes: the float cell differences are exact integers
// (checked: a tile whose cells spread over 2^23 or more raises the error flag).
// ---------------------------------------------------------------------------
constexpr int kReqPerWave = 64;

// Waves per SIMD the register allocation must allow (LDS allows the same).
constexpr int fused_min_waves(int P) { return P == 6 ? 5 : (P <= 8 ? 4 : (P == 12 ? 3 : 2)); }

template <int KIND, int P, bool SPARSE>
__global__ void __launch_bounds__(kBlock, fused_min_waves(P))
    k_step_fused(Tables t, SplitBuf in, SplitBuf out, Phys ph, int halo, int nsub) {
  constexpr int T = kBlock * P;
  constexpr int NW = kBlock / 64;
  constexpr int RQ = kReqPerWave;
  __shared__ float4 s_nodes[T];
  __shared__ int4 s_req[NW * (RQ + 1)];  // per wave: RQ requests, then one sink slot
  // End sites of each wave, double-buffered: [parity][cell, offset][slot][end],
  // wave w in slot w + 1.  A wave reaches its own and its neighbours' entries
  // through one LDS pointer held in a vector register, so every access is an
  // immediate offset of it (no per-access address moves); cells and offsets
  // are stored as single words, so no two registers need to be adjacent.
  __shared__ float s_edge[2][2][NW + 2][2];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = uniform_i32(tid >> 6);
  // The elastic constant and the time step are kept in vector registers:
  // on gfx950 a VALU instruction with a scalar-register operand issues more
  // slowly than its all-vector form (measured for an FP32 add: 0.24 against
  // 0.35 wave instructions per SIMD cycle), and every site update uses both.
  float cel = ph.cf, dt = ph.dtf;
  asm volatile("" : "+v"(cel));
  asm volatile("" : "+v"(dt));
  const float g = ph.sgn_strf;
  // Unit disorder strength (g = +1 for force values, -1 for potential
  // values): the service pass then forms the coefficients without the four
  // multiplications by g (exactly the same values).
  const bool unit_g = g == kind_sign<KIND>();
  lds_f32* eb = (lds_f32*)&s_edge[0][0][wv][0];  // slot wv: the left neighbour's entries
  asm volatile("" : "+v"(eb));
  // entry of parity `pa`, word q (0 cell, 1 offset), slot wv + ds, end e
  auto edge = [&](int pa, int q, int ds, int e) -> lds_f32& {
    return eb[((pa * 2 + q) * (NW + 2) + ds) * 2 + e];
  };

  for (int ti = blockIdx.x; ti < t.n_ft; ti += gridDim.x) {
    const int s = uniform_i32(t.ft_s[ti]);
    const int p0 = uniform_i32(t.ft_p0[ti]);
    const int len = uniform_i32(t.ft_len[ti]);
    const int L = uniform_i32(t.L[s]);
    const int64_t base = uniform_i64(t.off[s]);
    const uint32_t id = (uint32_t)uniform_i32((int)t.did[s]);
    const float f = t.f32[s];
    const int start = p0 - halo;
    int start_mod = start % L;
    if (start_mod < 0) start_mod += L;
    constexpr int VW = (P % 4 == 0) ? 4 : 2;  // sites per vector load / store
    const bool contiguous = start >= 0 && start + T <= L && (start % VW) == 0;
    // The tile crosses the end of its chain: only then does a site's column
    // need wrapping in the service pass.
    const bool wraps = start_mod + T > L;
    const int32_t cbase = uniform_i32(in.cell[base + start_mod]);

    float c[P];  // cell - cbase, an exact integer
    float r[P];
    float4 a[P];
    bool far = false;
    if (contiguous) {
      const int64_t gi = base + start + tid * P;
#pragma unroll
      for (int v = 0; v < P / VW; ++v) {
        int32_t cc[VW];
        float rr[VW];
        if constexpr (VW == 4) {
          const int4 cv = *reinterpret_cast<const int4*>(in.cell + gi + 4 * v);
          const float4 rv = *reinterpret_cast<const float4*>(in.frac + gi + 4 * v);
          cc[0] = cv.x; cc[1] = cv.y; cc[2] = cv.z; cc[3] = cv.w;
          rr[0] = rv.x; rr[1] = rv.y; rr[2] = rv.z; rr[3] = rv.w;
        } else {
          const int2 cv = *reinterpret_cast<const int2*>(in.cell + gi + 2 * v);
          const float2 rv = *reinterpret_cast<const float2*>(in.frac + gi + 2 * v);
          cc[0] = cv.x; cc[1] = cv.y;
          rr[0] = rv.x; rr[1] = rv.y;
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) {
          const int32_t d = cc[e] - cbase;
          far |= (uint32_t)(d + (1 << 23)) >= (1u << 24);
          c[VW * v + e] = (float)d;
          r[VW * v + e] = rr[e];
        }
      }
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const float4 nd = in.nodes[gi + i];
        s_nodes[i * kBlock + tid] = nd;
        a[i] = spline_coef<KIND>(nd.x, nd.y, nd.z, nd.w, g, f);
      }
    } else {
      int pos = (start_mod + tid * P) % L;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int32_t cc = in.cell[base + pos] - cbase;
        far |= (uint32_t)(cc + (1 << 23)) >= (1u << 24);
        c[i] = (float)cc;
        r[i] = in.frac[base + pos];
        const float4 nd = in.nodes[base + pos];
        s_nodes[i * kBlock + tid] = nd;
        a[i] = spline_coef<KIND>(nd.x, nd.y, nd.z, nd.w, g, f);
        pos = (pos + 1 == L) ? 0 : pos + 1;
      }
    }
    if (__ballot(far) && lane == 0) atomicOr(t.err, 1);
    if (lane == 0) {
      edge(0, 0, 1, 0) = c[0];
      edge(0, 1, 1, 0) = r[0];
    }
    if (lane == 63) {
      edge(0, 0, 1, 1) = c[P - 1];
      edge(0, 1, 1, 1) = r[P - 1];
    }
    __syncthreads();

    // One sub-step; the loop runs it twice per trip so that the state
    // arrays alternate between two register sets without copies.
    auto substep = [&](const int par) __attribute__((always_inline)) {
      // Neighbours of this thread's end sites.  The tile ends reflect.
      float cle = from_lower_lane(c[P - 1]);
      float rle = from_lower_lane(r[P - 1]);
      float cre = from_upper_lane(c[0]);
      float rre = from_upper_lane(r[0]);
      if (lane == 0) {
        if (wv > 0) {
          cle = edge(par, 0, 0, 1);
          rle = edge(par, 1, 0, 1);
        } else {
          cle = c[0];
          rle = r[0];
        }
      }
      if (lane == 63) {
        if (wv < NW - 1) {
          cre = edge(par, 0, 2, 0);
          rre = edge(par, 1, 2, 0);
        } else {
          cre = c[P - 1];
          rre = r[P - 1];
        }
      }

      // Wave priorities (s_setprio): a wave takes its steps and posts its
      // requests at the highest priority, serves and reads them back at the
      // lowest, and publishes its edges towards the barrier in between.  The
      // SIMD then issues the long, independent step chains first and fills
      // their gaps with the latency-bound request path of the other waves.
      __builtin_amdgcn_s_setprio(3);
      // Euler step of every site (Jacobi: old values of the neighbours); a
      // site that changed cell posts a request into this wave's region, at
      // byte offset kb[i] of s_req.  Requests past the region's RQ entries go
      // to its sink slot and are served by their own lane below.
      uint32_t kb[P];
      uint32_t nreq = 0u;  // wave-uniform
      const int rbase = wv * (RQ + 1);
      const uint32_t rbase_b = (uint32_t)rbase * (uint32_t)sizeof(int4);
      const uint32_t sink_b = rbase_b + (uint32_t)RQ * (uint32_t)sizeof(int4);
      float oc[P];          // cells before the step
      float dl = c[0] - cle;  // cell difference to the left neighbour
      float pr = rle;
      // All steps first (independent chains the scheduler can interleave),
      // then the requests of the sites that changed cell.
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const float nc = (i + 1 < P) ? c[i + 1] : cre;
        const float nr = (i + 1 < P) ? r[i + 1] : rre;
        const float dr = nc - c[i];
        const float lap = (dr - dl) + fmaf(-2.0f, r[i], pr + nr);
        const float F = fmaf(cel, lap, spline_eval<KIND>(a[i], r[i]));
        dl = dr;
        pr = r[i];
        oc[i] = c[i];
        c[i] = oc[i] + split_advance(r[i], F, dt);
      }
      // The sparse variant first checks whether any site of the wave changed
      // cell and skips the request bookkeeping when none did.
      bool book = true;
      if constexpr (SPARSE) {
        uint64_t any_move = 0u;
#pragma unroll
        for (int i = 0; i < P; ++i) any_move |= __ballot(c[i] != oc[i]);
        book = any_move != 0u;
      }
      if (book) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const bool mv = c[i] != oc[i];
        const uint64_t moved = __ballot(mv);
        const uint32_t cnt = (uint32_t)__popcll(moved);
        // The wave-uniform part stays one scalar operand of the address;
        // requests past the region land in its sink slot.
        kb[i] = min(mbcnt64(moved) * (uint32_t)sizeof(int4) +
                        (uint32_t)uniform_i32((int)(rbase_b + nreq * (uint32_t)sizeof(int4))),
                    sink_b);
        if (mv) {
          // The two cells go in the order of their registers, which swap
          // roles every sub-step: {new, old} on even sub-steps, {old, new}
          // on odd ones, so the three words stay one store without copies.
          const float w1 = par ? oc[i] : c[i];
          const float w2 = par ? c[i] : oc[i];
          *reinterpret_cast<int3*>(reinterpret_cast<char*>(s_req) + kb[i]) =
              make_int3(i * kBlock + tid, __float_as_int(w1), __float_as_int(w2));
        }
        nreq += cnt;
      }
      // Serve this wave's requests with this wave's lanes: lane q takes request
      // q.  The requests, their node windows and the replies belong to this
      // wave only, and a wave's LDS operations complete in program order, so
      // no workgroup barrier is needed between posting, serving and reading.
      __builtin_amdgcn_s_setprio(0);
      const uint32_t nserve = nreq < (uint32_t)RQ ? nreq : (uint32_t)RQ;
      if (nserve > 0u) {
        __builtin_amdgcn_wave_barrier();
        if ((uint32_t)lane < nserve) {
          const int slot = rbase + lane;
          const int4 rq = s_req[slot];  // {node index, cells (relative to cbase) in sub-step order}
          const int ni = rq.x;
          const float cnew = __int_as_float(par ? rq.z : rq.y);
          const float move = cnew - __int_as_float(par ? rq.y : rq.z);
          const int32_t cell = cbase + (int32_t)cnew;
          const int lp = (int)(((uint32_t)ni % kBlock) * P + (uint32_t)ni / kBlock);  // tile-local position
          int j = start_mod + lp;
          if (wraps) {
            if (j >= L) j -= L;
            if (j >= L) j %= L;
          }
          float4 w4 = s_nodes[ni];
          if (move == 1.0f) {
            w4 = make_float4(w4.y, w4.z, w4.w, node_f32<KIND>((uint32_t)j, cell + 2, id, ph.k0, ph.k1, ph.period));
          } else if (move == -1.0f) {
            w4 = make_float4(node_f32<KIND>((uint32_t)j, cell - 1, id, ph.k0, ph.k1, ph.period), w4.x, w4.y, w4.z);
          } else {
            w4 = make_float4(node_f32<KIND>((uint32_t)j, cell - 1, id, ph.k0, ph.k1, ph.period),
                             node_f32<KIND>((uint32_t)j, cell, id, ph.k0, ph.k1, ph.period),
                             node_f32<KIND>((uint32_t)j, cell + 1, id, ph.k0, ph.k1, ph.period),
                             node_f32<KIND>((uint32_t)j, cell + 2, id, ph.k0, ph.k1, ph.period));
          }
          s_nodes[ni] = w4;
          float4 co;
          if (unit_g) co = spline_coef<KIND>(w4.x, w4.y, w4.z, w4.w, kind_sign<KIND>(), f);
          else co = spline_coef<KIND>(w4.x, w4.y, w4.z, w4.w, g, f);
          s_req[slot] = make_int4(__float_as_int(co.x), __float_as_int(co.y), __float_as_int(co.z),
                                  __float_as_int(co.w));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      // Requesters read their new coefficients (a request past the region
      // reads its sink slot and is redone below); a wave without requests
      // skips the slot checks.
      if (nreq > 0u) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
          if (c[i] != oc[i]) {
            const int4 v = *reinterpret_cast<const int4*>(reinterpret_cast<const char*>(s_req) + kb[i]);
            a[i] = make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z),
                               __int_as_float(v.w));
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
      // Rare: more requests than the region holds (a burst of cell changes).
      // Those past it regenerate their window on their own lane.
      if (nreq > (uint32_t)RQ) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
          if (c[i] != oc[i] && kb[i] == sink_b) {
            int j = start_mod + tid * P;
            asm volatile("" : "+v"(j));  // keep this rare path's index arithmetic here
            j += i;
            if (j >= L) j -= L;
            if (j >= L) j %= L;
            const int32_t cell = cbase + (int32_t)c[i];
            const float4 w4 = make_float4(node_f32<KIND>((uint32_t)j, cell - 1, id, ph.k0, ph.k1, ph.period),
                                          node_f32<KIND>((uint32_t)j, cell, id, ph.k0, ph.k1, ph.period),
                                          node_f32<KIND>((uint32_t)j, cell + 1, id, ph.k0, ph.k1, ph.period),
                                          node_f32<KIND>((uint32_t)j, cell + 2, id, ph.k0, ph.k1, ph.period));
            s_nodes[i * kBlock + tid] = w4;
            a[i] = spline_coef<KIND>(w4.x, w4.y, w4.z, w4.w, g, f);
          }
        }
      }
      }  // book
      __builtin_amdgcn_s_setprio(2);
      // Publish this wave's end sites for the neighbouring waves' next sub-step.
      if (lane == 0) {
        edge(par ^ 1, 0, 1, 0) = c[0];
        edge(par ^ 1, 1, 1, 0) = r[0];
      }
      if (lane == 63) {
        edge(par ^ 1, 0, 1, 1) = c[P - 1];
        edge(par ^ 1, 1, 1, 1) = r[P - 1];
      }
      __syncthreads();
    };
    int sub = 0;
    for (; sub + 2 <= nsub; sub += 2) {
      substep(0);
      substep(1);
    }
    if (sub < nsub) substep(0);

    // Write the valid part: tile-local q in [halo, halo + len).
    int qb = tid * P;
    asm volatile("" : "+v"(qb));
    const int64_t g0 = base + p0 + (qb - halo);
    if (qb >= halo && qb + P <= halo + len && (g0 % VW) == 0) {
#pragma unroll
      for (int v = 0; v < P / VW; ++v) {
        if constexpr (VW == 4) {
          *reinterpret_cast<int4*>(out.cell + g0 + 4 * v) =
              make_int4(cbase + (int32_t)c[4 * v], cbase + (int32_t)c[4 * v + 1],
                        cbase + (int32_t)c[4 * v + 2], cbase + (int32_t)c[4 * v + 3]);
          *reinterpret_cast<float4*>(out.frac + g0 + 4 * v) =
              make_float4(r[4 * v], r[4 * v + 1], r[4 * v + 2], r[4 * v + 3]);
        } else {
          *reinterpret_cast<int2*>(out.cell + g0 + 2 * v) =
              make_int2(cbase + (int32_t)c[2 * v], cbase + (int32_t)c[2 * v + 1]);
          *reinterpret_cast<float2*>(out.frac + g0 + 2 * v) = make_float2(r[2 * v], r[2 * v + 1]);
        }
      }
#pragma unroll
      for (int i = 0; i < P; ++i) out.nodes[g0 + i] = s_nodes[i * kBlock + tid];
    } else {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        const int q = qb + i;
        if (q >= halo && q < halo + len) {
          const int64_t gi = base + p0 + (q - halo);
          out.cell[gi] = cbase + (int32_t)c[i];
          out.frac[gi] = r[i];
          out.nodes[gi] = s_nodes[i * kBlock + tid];
        }
      }
    }
    __syncthreads();  // s_nodes and s_edge are reused by the next tile
  }
}

// ---------------------------------------------------------------------------
// Measurement partials (Eqs. (3)-(5)) of the state at one step.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(kBlock)
    k_meas_plain(Tables t, const double* __restrict__ u, Phys ph, Partial* part) {
  __shared__ double lds[3 * (kBlock / 64)];
  const int tile = blockIdx.x;
  const int s = t.mt_s[tile];
  const int p0 = t.mt_p0[tile], len = t.mt_len[tile];
  const int L = t.L[s];
  const int64_t base = t.off[s];
  const uint32_t id = t.did[s];
  const double f = t.f[s];
  const PlainPhys pp{ph.c, ph.dt, ph.strength};
  const VectorKeys keys = vector_keys(ph.k0, ph.k1);
  const double K = u[base + p0];  // shift: the tile's first site (exactly 0 for a flat tile)
  double sf = 0.0, s1 = 0.0, s2 = 0.0;
  for (int q = threadIdx.x; q < len; q += kBlock) {
    const int j = p0 + q;
    const int jm = (j == 0) ? L - 1 : j - 1;
    const int jp = (j == L - 1) ? 0 : j + 1;
    const double uj = u[base + j];
    sf += plain_force<KIND>(u[base + jm], uj, u[base + jp], (uint32_t)j, id, keys, f, ph.period,
                            pp);
    const double x = uj - K;
    s1 += x;
    s2 += x * x;
  }
  block_sum3(sf, s1, s2, lds);
  if (threadIdx.x == 0) part[tile] = Partial{sf, s1, s2, K};
}

template <int KIND>
__global__ void __launch_bounds__(kBlock) k_meas_split(Tables t, SplitBuf b, Phys ph, Partial* part) {
  __shared__ double lds[3 * (kBlock / 64)];
  const int tile = blockIdx.x;
  const int s = t.mt_s[tile];
  const int p0 = t.mt_p0[tile], len = t.mt_len[tile];
  const int L = t.L[s];
  const int64_t base = t.off[s];
  const uint32_t id = t.did[s];
  const float f = t.f32[s];
  const SplitPhys sp{ph.cf, ph.dtf, ph.sgn_strf};
  const int32_t Kc = b.cell[base + p0];  // shift: the tile's first site
  const double Kr = (double)b.frac[base + p0];
  const VectorKeys keys = vector_keys(ph.k0, ph.k1);
  double sf = 0.0, s1 = 0.0, s2 = 0.0;
  for (int q = threadIdx.x; q < len; q += kBlock) {
    const int j = p0 + q;
    const int jm = (j == 0) ? L - 1 : j - 1;
    const int jp = (j == L - 1) ? 0 : j + 1;
    const int32_t c = b.cell[base + j];
    const float r = b.frac[base + j];
    float n0, n1, n2, n3;
    if (b.nodes) {  // the node cache of the fused path holds the same four values
      const float4 nd = b.nodes[base + j];
      n0 = nd.x;
      n1 = nd.y;
      n2 = nd.z;
      n3 = nd.w;
    } else {
      nodes_of<KIND>((uint32_t)j, c, id, ph, keys, n0, n1, n2, n3);
    }
    const float4 a = spline_coef<KIND>(n0, n1, n2, n3, sp.sgn_str, f);
    const float F = split_force<KIND>(c, r, b.cell[base + jm], b.frac[base + jm], b.cell[base + jp],
                                      b.frac[base + jp], a, sp.c);
    sf += (double)F;
    const double x = (double)(c - Kc) + ((double)r - Kr);  // exact
    s1 += x;
    s2 += x * x;
  }
  block_sum3(sf, s1, s2, lds);
  if (threadIdx.x == 0) part[tile] = Partial{sf, s1, s2, (double)Kc + Kr};
}

// Per-sample combine of tile partials: mean and sum of squared deviations by
// the pairwise update of Chan, Golub and LeVeque, in a fixed order.
struct Moments {
  double n, mean, m2, sf;
};

__device__ __forceinline__ Moments combine(const Moments& a, const Moments& b) {
  if (a.n == 0.0) return b;
  if (b.n == 0.0) return a;
  const double n = a.n + b.n;
  const double d = b.mean - a.mean;
  Moments r;
  r.n = n;
  r.mean = a.mean + d * (b.n / n);
  r.m2 = (a.m2 + b.m2) + d * d * (a.n * b.n / n);
  r.sf = a.sf + b.sf;
  return r;
}

__global__ void __launch_bounds__(kBlock)
    k_meas_final(Tables t, const Partial* part, int meas_index, int n_meas, double* series) {
  __shared__ Moments lds[kBlock];
  const int s = blockIdx.x;
  const int t0 = t.mt_first[s], t1 = t.mt_first[s + 1];
  Moments acc{0.0, 0.0, 0.0, 0.0};
  for (int ti = t0 + threadIdx.x; ti < t1; ti += kBlock) {
    const Partial p = part[ti];
    const double n = (double)t.mt_len[ti];
    Moments m;
    m.n = n;
    m.mean = p.shift + p.s1 / n;
    m.m2 = p.s2 - p.s1 * (p.s1 / n);
    m.sf = p.sum_f;
    acc = combine(acc, m);
  }
  lds[threadIdx.x] = acc;
  __syncthreads();
  for (int stride = kBlock / 2; stride >= 1; stride >>= 1) {
    if ((int)threadIdx.x < stride) lds[threadIdx.x] = combine(lds[threadIdx.x], lds[threadIdx.x + stride]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const Moments m = lds[0];
    const double L = (double)t.L[s];
    double* out = series + ((int64_t)s * n_meas + meas_index) * 3;
    out[0] = m.sf / L;
    out[1] = m.mean;
    out[2] = (m.m2 > 0.0 ? m.m2 : 0.0) / L;
  }
}

// Disorder average over samples of one measurement index per workgroup:
// two passes (mean, then squared deviations) in a fixed order.
__device__ __forceinline__ double block_sum1(double v, double* lds) {
  v = wave_sum_f64(v);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < kBlock / 64; ++i) s += lds[i];
  __syncthreads();
  return s;
}

__global__ void __launch_bounds__(kBlock)
    k_ensemble(int S, int n_meas, const double* __restrict__ series, double* __restrict__ out) {
  __shared__ double lds[kBlock / 64];
  const int mi = blockIdx.x;
  double mean[3], m2[3];
  for (int q = 0; q < 3; ++q) {
    double acc = 0.0;
    for (int s = threadIdx.x; s < S; s += kBlock) acc += series[((int64_t)s * n_meas + mi) * 3 + q];
    mean[q] = block_sum1(acc, lds) / (double)S;
    double dev = 0.0;
    for (int s = threadIdx.x; s < S; s += kBlock) {
      const double e = series[((int64_t)s * n_meas + mi) * 3 + q] - mean[q];
      dev += e * e;
    }
    m2[q] = block_sum1(dev, lds);
  }
  if (threadIdx.x == 0) {
    // series layout per sample: {v, ubar, w2}; output rows: v, se, w2, se, ubar, se, w2 about ensemble ubar
    const int src[3] = {0, 2, 1};
    for (int r = 0; r < 3; ++r) {
      const int q = src[r];
      out[(2 * r) * n_meas + mi] = mean[q];
      out[(2 * r + 1) * n_meas + mi] = S > 1 ? sqrt(m2[q] / (double)(S - 1) / (double)S) : 0.0;
    }
    out[6 * n_meas + mi] = mean[2] + m2[1] / (double)S;
  }
}

__global__ void k_fill_i32(int* p, int64_t n, int value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ void k_fill_f64(double* p, int64_t n, double value) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = value;
}

// ---------------------------------------------------------------------------
// Debug kernels.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
    k_philox_fill(const uint4* __restrict__ ctr, uint32_t k0, uint32_t k1, uint4* __restrict__ out,
                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  uint4 x = ctr[i];
  philox4x32_10(x.x, x.y, x.z, x.w, k0, k1);
  out[i] = x;
}

template <int KIND>
__global__ void __launch_bounds__(kBlock)
    k_force_eval(double strength, uint32_t k0, uint32_t k1, int32_t period, int precision,
                 const uint32_t* __restrict__ did, const int32_t* __restrict__ jj,
                 const int32_t* __restrict__ cell, const double* __restrict__ frac,
                 double* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = (uint32_t)jj[i];
  const uint32_t id = did[i];
  if (precision == 0) {
    const double u = (double)cell[i] + frac[i];
    const double nf = floor(u);
    const int32_t c = (int32_t)nf;
    double p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = strength * node_f64<KIND>(j, c - 1 + q, id, k0, k1, period);
    out[i] = spline_f64<KIND>(p, u - nf);
  } else {
    const int32_t c = cell[i];
    const float r = (float)frac[i];
    const float p0 = node_f32<KIND>(j, c - 1, id, k0, k1, period);
    const float p1 = node_f32<KIND>(j, c, id, k0, k1, period);
    const float p2 = node_f32<KIND>(j, c + 1, id, k0, k1, period);
    const float p3 = node_f32<KIND>(j, c + 2, id, k0, k1, period);
    const float sg = kind_sign<KIND>() * (float)strength;
    out[i] = (double)spline_eval<KIND>(spline_coef<KIND>(p0, p1, p2, p3, sg, 0.0f), r);
  }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
#define QEW_KIND_DISPATCH(kind, KERNEL, ...)                      \
  do {                                                            \
    switch (kind) {                                               \
      case kRF: hipLaunchKernelGGL(KERNEL<kRF>, __VA_ARGS__); break;       \
      case kRB: hipLaunchKernelGGL(KERNEL<kRB>, __VA_ARGS__); break;       \
      case kRBLin: hipLaunchKernelGGL(KERNEL<kRBLin>, __VA_ARGS__); break; \
      default: hipLaunchKernelGGL(KERNEL<kRFPc>, __VA_ARGS__); break;      \
    }                                                             \
  } while (0)

hipError_t launch_init_plain(const Tables& t, double* u, hipStream_t st) {
  hipLaunchKernelGGL(k_init_plain, dim3(t.n_mt), dim3(kBlock), 0, st, t, u);
  return hipGetLastError();
}

hipError_t launch_init_split(const Tables& t, SplitBuf b, const Phys& ph, int kind, bool nodes,
                             hipStream_t st) {
  QEW_KIND_DISPATCH(kind, k_init_split, dim3(t.n_mt), dim3(kBlock), 0, st, t, b, ph, nodes ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_refresh_nodes(const Tables& t, SplitBuf b, const Phys& ph, int kind,
                                hipStream_t st) {
  QEW_KIND_DISPATCH(kind, k_refresh_nodes, dim3(t.n_mt), dim3(kBlock), 0, st, t, b, ph);
  return hipGetLastError();
}

template <int KIND>
static void launch_plain_kind(const Tables& t, const double* uin, double* uout, const Phys& ph,
                              Partial* part, hipStream_t st) {
  if (part) hipLaunchKernelGGL((k_step_plain<KIND, true>), dim3(t.n_mt), dim3(kBlock), 0, st, t, uin, uout, ph, part);
  else hipLaunchKernelGGL((k_step_plain<KIND, false>), dim3(t.n_mt), dim3(kBlock), 0, st, t, uin, uout, ph, part);
}

hipError_t launch_step_plain(const Tables& t, const double* uin, double* uout, const Phys& ph,
                             int kind, Partial* part, hipStream_t st) {
  switch (kind) {
    case kRF: launch_plain_kind<kRF>(t, uin, uout, ph, part, st); break;
    case kRB: launch_plain_kind<kRB>(t, uin, uout, ph, part, st); break;
    case kRBLin: launch_plain_kind<kRBLin>(t, uin, uout, ph, part, st); break;
    default: launch_plain_kind<kRFPc>(t, uin, uout, ph, part, st); break;
  }
  return hipGetLastError();
}

template <int KIND>
static void launch_split1_kind(const Tables& t, SplitBuf in, SplitBuf out, const Phys& ph,
                               Partial* part, hipStream_t st) {
  if (part) hipLaunchKernelGGL((k_step_split1<KIND, true>), dim3(t.n_mt), dim3(kBlock), 0, st, t, in, out, ph, part);
  else hipLaunchKernelGGL((k_step_split1<KIND, false>), dim3(t.n_mt), dim3(kBlock), 0, st, t, in, out, ph, part);
}

hipError_t launch_step_split1(const Tables& t, SplitBuf in, SplitBuf out, const Phys& ph, int kind,
                              Partial* part, hipStream_t st) {
  switch (kind) {
    case kRF: launch_split1_kind<kRF>(t, in, out, ph, part, st); break;
    case kRB: launch_split1_kind<kRB>(t, in, out, ph, part, st); break;
    case kRBLin: launch_split1_kind<kRBLin>(t, in, out, ph, part, st); break;
    default: launch_split1_kind<kRFPc>(t, in, out, ph, part, st); break;
  }
  return hipGetLastError();
}

template <int KIND, int P>
static const void* fused_ptr() {
  return reinterpret_cast<const void*>(&k_step_fused<KIND, P, false>);
}

static const void* fused_fn(int tile) {
  switch (tile) {
    case 1024: return fused_ptr<kRF, 4>();
    case 1536: return fused_ptr<kRF, 6>();
    case 2048: return fused_ptr<kRF, 8>();
    case 3072: return fused_ptr<kRF, 12>();
    default: return fused_ptr<kRF, 16>();
  }
}

int fused_max_grid(int tile) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn = fused_fn(tile);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess) return 0;
  if (per_cu < 1) per_cu = 1;
  return cus * per_cu;
}

bool fused_fits(int tile) {
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return false;
  hipFuncAttributes attr{};
  const void* fn = fused_fn(tile);
  if (hipFuncGetAttributes(&attr, fn) != hipSuccess) return false;
  return (int)attr.sharedSizeBytes <= max_lds;
}

template <int KIND, bool SPARSE>
static void launch_fused_kind(const Tables& t, SplitBuf in, SplitBuf out, const Phys& ph, int tile,
                              int halo, int nsub, dim3 g, dim3 b, hipStream_t st) {
  if (tile == 1024) hipLaunchKernelGGL((k_step_fused<KIND, 4, SPARSE>), g, b, 0, st, t, in, out, ph, halo, nsub);
  else if (tile == 1536) hipLaunchKernelGGL((k_step_fused<KIND, 6, SPARSE>), g, b, 0, st, t, in, out, ph, halo, nsub);
  else if (tile == 2048) hipLaunchKernelGGL((k_step_fused<KIND, 8, SPARSE>), g, b, 0, st, t, in, out, ph, halo, nsub);
  else if (tile == 3072) hipLaunchKernelGGL((k_step_fused<KIND, 12, SPARSE>), g, b, 0, st, t, in, out, ph, halo, nsub);
  else hipLaunchKernelGGL((k_step_fused<KIND, 16, SPARSE>), g, b, 0, st, t, in, out, ph, halo, nsub);
}

template <bool SPARSE>
static void launch_fused_variant(const Tables& t, SplitBuf in, SplitBuf out, const Phys& ph, int kind,
                                 int tile, int halo, int nsub, dim3 g, dim3 b, hipStream_t st) {
  switch (kind) {
    case kRF: launch_fused_kind<kRF, SPARSE>(t, in, out, ph, tile, halo, nsub, g, b, st); break;
    case kRB: launch_fused_kind<kRB, SPARSE>(t, in, out, ph, tile, halo, nsub, g, b, st); break;
    case kRBLin: launch_fused_kind<kRBLin, SPARSE>(t, in, out, ph, tile, halo, nsub, g, b, st); break;
    default: launch_fused_kind<kRFPc, SPARSE>(t, in, out, ph, tile, halo, nsub, g, b, st); break;
  }
}

hipError_t launch_step_fused(const Tables& t, SplitBuf in, SplitBuf out, const Phys& ph, int kind,
                             int tile, int halo, int nsub, int grid, bool sparse, hipStream_t st) {
  const dim3 g(grid), b(kBlock);
  if (sparse) launch_fused_variant<true>(t, in, out, ph, kind, tile, halo, nsub, g, b, st);
  else launch_fused_variant<false>(t, in, out, ph, kind, tile, halo, nsub, g, b, st);
  return hipGetLastError();
}

hipError_t launch_meas_plain(const Tables& t, const double* u, const Phys& ph, int kind,
                             Partial* part, hipStream_t st) {
  QEW_KIND_DISPATCH(kind, k_meas_plain, dim3(t.n_mt), dim3(kBlock), 0, st, t, u, ph, part);
  return hipGetLastError();
}

hipError_t launch_meas_split(const Tables& t, SplitBuf b, const Phys& ph, int kind, Partial* part,
                             hipStream_t st) {
  QEW_KIND_DISPATCH(kind, k_meas_split, dim3(t.n_mt), dim3(kBlock), 0, st, t, b, ph, part);
  return hipGetLastError();
}

hipError_t launch_meas_final(const Tables& t, int n_samples, const Partial* part, int meas_index,
                             int n_meas, double* series, hipStream_t st) {
  hipLaunchKernelGGL(k_meas_final, dim3(n_samples), dim3(kBlock), 0, st, t, part, meas_index, n_meas,
                     series);
  return hipGetLastError();
}

hipError_t launch_ensemble(int n_samples, int n_meas, const double* series, double* out,
                           hipStream_t st) {
  if (n_meas <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ensemble, dim3(n_meas), dim3(kBlock), 0, st, n_samples, n_meas, series, out);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t n, int value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((uint32_t)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p, n,
                     value);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((uint32_t)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p, n,
                     value);
  return hipGetLastError();
}

hipError_t launch_philox_fill(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                              int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_philox_fill, dim3((uint32_t)blocks), dim3(kBlock), 0, st,
                     reinterpret_cast<const uint4*>(ctr), k0, k1, reinterpret_cast<uint4*>(out), n);
  return hipGetLastError();
}

hipError_t launch_force_eval(int kind, double strength, uint32_t k0, uint32_t k1, int32_t period,
                             int precision, const uint32_t* did, const int32_t* j,
                             const int32_t* cell, const double* frac, double* out, int64_t n,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  QEW_KIND_DISPATCH(kind, k_force_eval, dim3((uint32_t)blocks), dim3(kBlock), 0, st, strength, k0, k1,
                    period, precision, did, j, cell, frac, out, n);
  return hipGetLastError();
}

}  // namespace qew
