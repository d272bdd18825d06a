// Internal types and kernel launchers of the gtod library (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gtod {

// Frequency axis padded to a multiple of the contraction depth chunk, the
// channel axis to a multiple of the 32-wide MFMA tile.
constexpr int kFPad = 32;
constexpr int kKPad = 32;
// Rows of one contraction tile (time samples of one pixel) and of one
// panel block.  A pixel's rows inside a chunk are padded to kRowPad.
constexpr int kRowPad = 128;
constexpr int kPanelRows = 32;

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Everything the panel kernel needs for one chunk of rows.
// Rows of the chunk: r = pl * Tpad + tl for local pixel pl in [0, n_pix)
// and local sample tl in [0, Tpad); a row is valid when tl < Tc; its
// absolute sample is t0 + tl and its job pixel is p0 + pl.
struct PanelArgs {
  const float* tau;      // [n_pwv][Fp] zenith optical depth
  const float* E;        // [Fp] emission with a transparent sky
  const float* D;        // [Fp] coefficient of the sky emissivity
  const float* W;        // [Fp] gain on the source
  const float* Pref;     // [Fp] reference spectrum
  int F, Fp, n_pwv;
  double pwv0, dpwv;
  const double* scr;     // [ny][nx]
  int64_t nx, ny;
  double dx, dy, ix0, iy0, h, wind;
  int scan_kind;
  double phi0, theta0, r_petal, omega, Omega;
  const double* traj;    // [t_total][2]
  double f_s;
  const double* dphi;    // [n_pix_job] device
  const double* dtheta;
  int p0, n_pix;
  const float* cube;     // [n_el][n_az][cube_ld] or null
  int n_az, n_el;
  int64_t cube_ld;
  double az0, daz, el0, del;
  int64_t t0;
  int Tc, Tpad;
  float* panel;          // [n_pix*Tpad][Fp]
  float* pwv_out;        // [n_pix_job][out_ld] or null
  int64_t out_t0, out_ld;
  unsigned long long* counters;  // [2]
  // Row order.  With a source cube the rows are processed grouped by the
  // source cell they read (a counting sort on key = coarse cell, last
  // bucket = no source), so that rows sharing cube corners run together.
  void* rinfo;           // [n_pix*Tpad] per-row quantities (RowInfo)
  uint32_t* key;         // [n_pix*Tpad] bucket of each row
  uint32_t* order;       // [n_pix*Tpad] rows grouped by bucket
  uint32_t* hist;        // [n_buckets] counts, then running offsets
  int n_buckets;         // coarse cells + 1; 1 = no sort
  int cell_shift;        // coarse cell = (el cell >> s, az cell >> s)
  int n_az_coarse;
};
constexpr int kPanelRowInfoBytes = 48;   // sizeof(RowInfo) rounded up
constexpr int kPanelMaxBuckets = 1 << 16;

struct GemmArgs {
  const float* panel;    // [rows][Fp] deviations dP
  const float* B;        // [3][Kp][Fp] B0, B1', B2 (fp32)
  const uint16_t* Bh;    // [3][Kp][Fp] bf16 hi
  const uint16_t* Bl;    // [3][Kp][Fp] bf16 lo
  const uint16_t* Bt;    // split responses tiled for the BF16 kernel
  const double* c0;      // [Kp] reference P_KID
  const double* c1;      // [Kp] reference NEP^2
  int Fp, K, Kp;
  int p0, n_pix, Tc, Tpad;
  int64_t t0, out_t0, out_ld;
  float fs_half;
  // The panel carries spectral powers times 2^pexp (power-of-two scale,
  // exact) so that dP and dP^2 stay in the normal FP32 range; the
  // epilogue multiplies by pinv = 2^-pexp.
  double pinv;
  float pinv_f;
  uint32_t key0, key1;
  int pix0;              // noise-key index of the job's pixel 0
  int photon, accumulate;
  // brightness-temperature output: tod = (P - kel_a) * kel_ib per channel
  int kelvin;
  const double* kel_a;   // [K]
  const double* kel_ib;  // [K]
  float* tod;
  float* p_kid;
  float* sigma;
  int n_tt;              // 128-row time tiles of the chunk
  int n_cg;              // channel groups (set by each contraction launcher)
};

struct PinkArgs {
  int64_t s0;            // first series of the batch (series = p*K + k)
  int n_series;
  int K;
  int M, M1, M2, lgM1, lgM2, N;
  double fs;
  float2* scratch;       // [n_series][M1][M2]
  const float* scale;    // [K] sqrt(A_k N fs / 4) / N
  const float* alpha;    // [K]
  uint32_t key0, key1;
  int pix0;              // noise-key index of the job's pixel 0
  float* tod;
  int64_t t_total, out_ld;
  int accumulate;
  int lgB2;              // log2 of the columns per pass-2 workgroup
  const float2* tab;     // [4096] e^{2 pi i m / 4096}
  float2* tab_w;         // the same table, written by k_pink_tables
};
constexpr int kPinkLgM2 = 11;                // log2 of the usual 1/f pass-1 length
constexpr int kPinkLgB2 = 4;                 // log2 of the 1/f pass-2 columns per workgroup
constexpr int kPinkTableFloat2 = 2 * 4096;   // reserved at the workspace head

// setup kernels (FP64)
struct SpecSetupArgs {
  int F, Fp, K, Kp, n_pwv, n_pass, mode;
  const double* nu;      // [F]
  const double* w;       // [F]
  const double* eta_z;   // [n_pwv][F]
  const double* pass_eta;   // [n_pass][F]
  const int* pass_kind;     // [n_pass]: 0 fixed temperature, 1 sky
  const double* pass_T;     // [n_pass]
  const double* f_hz; const double* R; const double* eta_peak;  // [K]
  const int* order;         // [K] upstream order (filterbank)
  const double* eta_filt;   // [F][K] (matrix mode)
  double t_atm, t_cmb, eta_taper, rho_surf, eta_pol, delta_J, eta_pb;
  double ref_pwv, pwv0, dpwv, ref_el;
  // outputs
  float* tau; float* E; float* D; float* W; float* Pref;
  double* tau64;            // [n_pwv][F] zenith optical depth, FP64
  double* E64; double* D64; // [F] cascade terms, FP64, unscaled
  double* Pref64;           // [Fp] the FP32 reference widened (exact)
  double* B0_64;            // [F][K] B0 = w eta, FP64
  double* B64;              // [2][F][K] scratch (B1, B2)
  float* B;                 // [3][Kp][Fp]
  uint16_t* Bh; uint16_t* Bl;
  double* c0; double* c1;   // [Kp]
};

// Optics passes after the atmosphere.  type: 0 eta from pool[off + j],
// 1 constant prm[0], 2 Ohmic (eps_ref, nu_ref), 3 dielectric absorption
// (d, n, tan delta), 4 dielectric surface (n).  coupling: 0 to P_JN(T),
// 1 to the sky.
struct PassTable {
  int n;
  const int* type;
  const int* coupling;
  const int* off;
  const double* prm;   // [n][3]
  const double* T;
  const double* pool;
};

// Skydip (brightness-temperature scale): a sweep of n zenith PWV values at
// one elevation, no source.
struct SkydipArgs {
  int F, K, n_pwv, n;
  double pwv_lo, pwv_hi, pwv0, dpwv, csc, t_atm;
  const double* tau64;   // [n_pwv][F]
  const double* E64;     // [F]
  const double* D64;     // [F]
  const double* B0;      // [F][K]
  double* Pm;            // [n][F] scratch: spectral power of each sweep row
  double* Xm;            // [n][F] scratch: sky emissivity 1 - eta_atm
  double* p_kid;         // [n][K]
  double* t_b;           // [n][K]
  double* a;             // [K] intercept
  double* b;             // [K] slope
  double* ib;            // [K] 1 / slope
};

void launch_skydip(const SkydipArgs& a, hipStream_t s);

// Common-mode subtraction and gridding of a Kelvin TOD (one channel group
// [k0, k0 + kg) per launch of the group kernels).
constexpr int kMaxMapN = 48;
struct ReduceArgs {
  int P, K, F, n_pwv;
  int64_t T, t0, ld;          // the TOD holds samples [t0, t0 + T), stride ld
  int k0, kg;
  int scan_kind;
  double r_petal, omega, Omega, f_s, theta0;
  const double* traj;         // [t_total][2]
  const double* dphi;         // [P] device (staged)
  const double* dtheta;       // [P]
  const int* off;             // [P] 1 if the spaxel is off source
  int n_out;
  const double* tau64;        // [n_pwv][F]
  const double* B0;           // [F][K]
  double pwv0, dpwv;
  const float* pwv;           // [P][pwv_ld] zenith PWV output, or null
  int64_t pwv_ld, pwv_len;
  double pwv_host;            // used when pwv is null
  double* pwv_mean;           // scratch [1]
  double* lnz;                // scratch [K] ln of the channel zenith transmission
  double2* scan_tab;          // scratch [T] (phi, theta)
  const float* tod;           // [P][K][ld] brightness temperature
  float* t_star;              // [P][K][ld] or null
  double* M;                  // scratch [kg][T] common-mode term
  int map_n;                  // 0: no maps
  double half, dcell;
  double2* stats;             // scratch [P][kg][C] (weight, mean)
  double* map;                // [K][C]
  double* weight;             // [K][C]
};

// Input preparation (section 2.2).
struct BeamArgs {
  int n_nodes;               // Gauss-Legendre nodes on [0, R_tel]
  double* gl_x;              // [n_nodes] scratch: nodes on [0, 1]
  double* gl_w;              // [n_nodes] weights on [0, 1]
  double r_tel, t_edge_db;
  const double* nu;          // [F] device
  int F, n_a, n_b;
  double da, db;             // grid spacings (rad) along a and b
  float* table;              // [F][n_b][n_a] peak-normalised far field
};
struct SrcConvArgs {
  const float* in;           // [n_el][n_az][ld_in] specific intensity
  int64_t ld_in, ld_out;
  int n_az, n_el, f0, nf;    // frequencies [f0, f0 + nf) of this batch
  double el0, del, scale;    // scale = A_p daz del
  const float* table;        // [nf][n_el][n_az] far field of the batch
  float* out;                // [n_el][n_az][ld_out]
};
struct ScreenConvArgs {
  const double* in;          // [ny][nx]
  double* out;
  int64_t nx, ny;
  int rx, ry;                // footprint half widths in cells
  double dx, dy, r_tel, t_edge_db;
  double* w;                 // [2ry+1][2rx+1] scratch: normalised weights
};
constexpr int kScreenTileX = 64, kScreenTileY = 32, kMaxFootprint = 32;
constexpr int kMaxSrcNodes = 20000;   // n_az n_el of a source grid
void launch_gauss_legendre(double* x, double* w, int n, hipStream_t s);
void launch_beam_table(const BeamArgs& a, hipStream_t s);
int launch_source_conv(const SrcConvArgs& a, hipStream_t s);   // 0 ok
void launch_screen_weights(const ScreenConvArgs& a, hipStream_t s);
int launch_screen_conv(const ScreenConvArgs& a, hipStream_t s); // 0 ok

// Context services for library parts outside the runtime file: device
// memory charged to the context's budget, the error message, and a few
// properties.  (The context type is defined by the runtime.)
}  // namespace gtod
struct gtod_ctx;
namespace gtod {
int32_t ctx_alloc(gtod_ctx* c, void** p, size_t bytes);
void ctx_free(gtod_ctx* c, void* p);
int32_t ctx_fail(gtod_ctx* c, int32_t status, const char* msg);
int ctx_device(const gtod_ctx* c);
double ctx_f_sample(const gtod_ctx* c);
int ctx_spec_channels(const gtod_ctx* c, int32_t spec_id);  // -1 if unknown
// Two library-owned streams (default priority) kept until the context is
// freed; null if creation failed.
hipStream_t ctx_sink_stream(gtod_ctx* c, int which);

void launch_reduce_setup(const ReduceArgs& a, hipStream_t s);
void launch_reduce_common(const ReduceArgs& a, hipStream_t s);
int launch_reduce_grid(const ReduceArgs& a, hipStream_t s);  // 0 ok
void launch_reduce_combine(const ReduceArgs& a, hipStream_t s);
void launch_spec_setup(const SpecSetupArgs& a, const PassTable& pt,
                       hipStream_t s);
void launch_scale_spectra(float* E, float* D, float* W, float* Pref, int Fp,
                          float scale, hipStream_t s);
void launch_panel(const PanelArgs& a, hipStream_t s);
void launch_gemm_f32(const GemmArgs& a, hipStream_t s);
void launch_gemm_bf16(const GemmArgs& a, hipStream_t s);
// Bytes of the tiled split responses of a Kp x Fp setup, and the kernel
// that builds them from the hi / lo planes.
size_t split_tiled_bytes(int Kp, int Fp);
void launch_tile_split_responses(const uint16_t* Bh, const uint16_t* Bl, uint16_t* Bt,
                                 int Kp, int Fp, float b2_scale, hipStream_t s);
void launch_pink_tables(const PinkArgs& a, hipStream_t s);
void launch_pink_pass1(const PinkArgs& a, hipStream_t s);
void launch_pink_pass2(const PinkArgs& a, hipStream_t s);
void launch_philox(const uint32_t* ctr, uint32_t* out, int64_t n,
                   uint32_t k0, uint32_t k1, hipStream_t s);

}  // namespace gtod
