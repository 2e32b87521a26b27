// qew_internal.hpp -- interface between the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qew {

// Device-resident tables of a plan (all pointers into the workspace).
struct Tables {
  const int64_t* off;       // [S] first site of sample s in a state buffer
  const int32_t* L;         // [S] chain length
  const double* f;          // [S] drive (FP64 path)
  const float* f32;         // [S] drive rounded to FP32 (split path)
  const uint32_t* did;      // [S] disorder id
  const int32_t* mt_s;      // [n_mt] measurement / one-step tiles: sample
  const int32_t* mt_p0;     //        first site
  const int32_t* mt_len;    //        sites
  const int32_t* mt_first;  // [S+1] first measurement tile of each sample
  const int32_t* ft_s;      // [n_ft] fused workgroup tiles: sample
  const int32_t* ft_p0;     //        first valid site
  const int32_t* ft_len;    //        valid sites
  int32_t n_mt;
  int32_t n_ft;
  int* err;                 // error flags raised by kernels (bit 0: tile cell span >= 2^23)
};

struct SplitBuf {
  int32_t* cell;   // [padded sites] integer part of u
  float* frac;     // [padded sites] u - cell in [0, 1)
  float4* nodes;   // [padded sites] nodes cell-1 .. cell+2 of each site (fused path only)
};

struct Phys {
  double c, dt, strength;
  float cf, dtf, sgn_strf;  // FP32 copies; sgn_strf = +strength (force values) or -strength (potential)
  uint32_t k0, k1;          // Philox key (seed words)
  int32_t period;           // transverse period of the disorder in u (0: none)
};

// Measurement partial of one tile: sum of F, sum of (u - K), sum of (u - K)^2, K.
struct Partial {
  double sum_f, s1, s2, shift;
};

constexpr int kMeasTile = 4096;   // sites per measurement / one-step tile
constexpr int kBlock = 256;       // threads per workgroup of every kernel
constexpr int kMaxHalo = 128;

// Launchers (return the launch error; all asynchronous on `st`).
hipError_t launch_init_plain(const Tables& t, double* u, hipStream_t st);
hipError_t launch_init_split(const Tables& t, SplitBuf b, const Phys& ph, int kind, bool nodes,
                             hipStream_t st);
hipError_t launch_refresh_nodes(const Tables& t, SplitBuf b, const Phys& ph, int kind,
                                hipStream_t st);
// One Euler step of every site; with `part` non-null the same launch also
// writes the measurement partials of the input state (the partials
// launch_meas_* would write, bit for bit).
hipError_t launch_step_plain(const Tables& t, const double* uin, double* uout, const Phys& ph,
                             int kind, Partial* part, hipStream_t st);
hipError_t launch_step_split1(const Tables& t, SplitBuf in, SplitBuf out, const Phys& ph, int kind,
                              Partial* part, hipStream_t st);
// `sparse`: the variant that skips the request bookkeeping of a wave whose
// sites did not change cell (for pinned or slow lines).
hipError_t launch_step_fused(const Tables& t, SplitBuf in, SplitBuf out, const Phys& ph, int kind,
                             int tile, int halo, int nsub, int grid, bool sparse, hipStream_t st);
int fused_max_grid(int tile);
bool fused_fits(int tile);  // static LDS of the tile's kernel within the device limit
hipError_t launch_meas_plain(const Tables& t, const double* u, const Phys& ph, int kind,
                             Partial* part, hipStream_t st);
// Split state: b.nodes non-null means it holds the four nodes of every
// site's current cell (the fused path's cache), which are then read instead
// of regenerated.
hipError_t launch_meas_split(const Tables& t, SplitBuf b, const Phys& ph, int kind, Partial* part,
                             hipStream_t st);
hipError_t launch_meas_final(const Tables& t, int n_samples, const Partial* part, int meas_index,
                             int n_meas, double* series, hipStream_t st);
hipError_t launch_ensemble(int n_samples, int n_meas, const double* series, double* out,
                           hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t n, double value, hipStream_t st);
hipError_t launch_fill_i32(int* p, int64_t n, int value, hipStream_t st);
hipError_t launch_philox_fill(const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out,
                              int64_t n, hipStream_t st);
hipError_t launch_force_eval(int kind, double strength, uint32_t k0, uint32_t k1, int32_t period,
                             int precision,
                             const uint32_t* did, const int32_t* j, const int32_t* cell,
                             const double* frac, double* out, int64_t n, hipStream_t st);

// Critical force and configuration of samples periodic in u (one workgroup
// per sample, the whole bisection in one launch).  u_io [S][L]: start in,
// last pinned configuration out; f_out [S][2]: the final bracket; st_out
// [S][2]: status (0 done, 1 no pinned configuration at the lower drive, 2 a
// trial undecided within max_sweeps, 3 out of rounds) and sweeps made.
struct CritParams {
  int32_t L, period, max_rounds;
  uint32_t k0, k1;
  double c, strength, f_lo, f_hi, tol_f, tol_force;
  int64_t max_sweeps;
};
constexpr int kCritMaxL = 4096;
size_t critical_lds_bytes(int L);
hipError_t launch_critical(int kind, const CritParams& q, int n_samples, const uint32_t* did, double* u_io,
                           double* f_out, int64_t* st_out, hipStream_t st);

// Structure factor at one measurement: pack, FFT passes, per-mode |U_n/L|^2,
// binned mean over samples into out[n_bins].  Every L_s equals L (power of
// two, at least 8); u_plain != nullptr selects the FP64 state, else `split`.
// The bins are cut into n_chunks chunks of modes [chunk_lo[c], chunk_lo[c+1])
// (bin b owns chunks chunk_first[b] .. chunk_first[b+1]-1); `part` holds one
// partial sum per chunk.
hipError_t launch_sq(const int64_t* off, int S, int64_t L, const double* u_plain, SplitBuf split,
                     double2* bufA, double2* bufB, const int32_t* chunk_lo, int n_chunks,
                     const int32_t* chunk_first, int n_bins, double* part, double* out,
                     hipStream_t st);

}  // namespace qew
