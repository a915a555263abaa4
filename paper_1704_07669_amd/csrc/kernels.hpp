// Host-side launchers of the device kernels (one translation unit per kernel family).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.hpp"

namespace sk {

// ---------------------------------------------------------------- test matrix Omega (Alg. 4 step 3)
hipError_t launch_omega_philox(uint64_t seed, int64_t n, int l, double* om64, int64_t ldo,
                               hipStream_t s);
hipError_t launch_omega_user(const double* src, int64_t ld, int64_t n, int l, double* om64,
                             int64_t ldo, hipStream_t s);
// Rounds Omega (column-major, l columns of length n, ld = NP) to the operand format of `mode`,
// writing the operand copy `omc` (LP x NP, zero padded) and replacing om64 by Omega' in FP64.
hipError_t launch_omega_quantize(int mode, int64_t n, int64_t NP, int l, int LP, double* om64,
                                 void* omc, hipStream_t s);
hipError_t launch_philox_words(uint64_t seed, uint64_t first, int64_t count, uint64_t* out,
                               hipStream_t s);

// ---------------------------------------------------------------- streaming pass (Alg. 4 steps 5-7)
// One row block of one stream as the streaming kernels see it.  A launch processes a group of such
// items (one for a single handle; one block each of several streams in a grouped serving launch);
// every workgroup finds its item by its first-workgroup offsets wg1 / wg2 / wgr.  The launch
// parameters of an item (split counts, strips) depend only on the item, so a block gives the same
// bits alone and in any group.
struct PassItem {
  const void* A;       // nrows x n row-major block (storage format of the group's src)
  int64_t lda;         // elements
  int64_t n;
  const void* omc;     // Omega' operand copy, LP x NP column-major
  int64_t NP;
  void* P1;            // split partials of g = a Omega: splits x LP x ldp
  int64_t ldp;         // row stride of P1 and Gop (>= nrows)
  int64_t kchunk;      // columns per split (multiple of 512)
  void* G;             // G, LP x ldg column-major (FP64 in F64 mode, FP32 otherwise)
  int64_t ldg;
  int64_t g_row0;      // first row of this block in G
  void* Gop;           // block-local operand copy of g for a^T g: LP x ldp (FP64 / FP32), or two
                       // LP x ldp BF16 arrays (hi, lo) in the BF16-operand modes
  double* H;           // H, LP x ldh column-major, FP64
  int64_t ldh;
  const int* fp8_exp;  // device exponent e of the block scale 2^e (FP8 mode), else null
  Ctrl* ctrl;
  int* nf_host;        // host-mapped flag also set when the block is non-finite (or null), so the
                       //   host sees it without waiting for the stream
  void* P2;            // row-split partials of a^T g: strips x rsplit x LP x strip width
  unsigned* counters;  // one zero-initialised arrival counter per strip
  int32_t nrows, vec_ok, splits, row_tiles;
  int32_t strips, rsplit, rchunk, red_wgs;
  int32_t wg1, wg2, wgr, wgh;   // first workgroup of the item in the g, a^T g, reduce and
                                //   row-split sum grids
  int32_t hsum_wgs;
  int32_t sum_col;     // G-operand column set to ones, so a^T g also accumulates the column sums
                       //   of a in that column of H (implicit centring); 0: none (column 0 is
                       //   always a sketch column)
  int32_t pad1, pad2;
};
struct PassGroup {
  int mode;            // Mode
  int src;             // sketch_dtype of the rows read by the kernels (F64/F32/BF16, or FP8 for
                       // pre-quantised staging); one format per group
  int LP;              // l rounded up to 16
  int NT;              // LP / 16
  int count;           // items
  PassItem one;        // the item when count == 1 (passed by value)
  const PassItem* dev; // device copy of the items when count > 1
  int64_t wg1_total, wg2_total, wgr_total, wgh_total;
};
constexpr int kNpAlign = 512;        // n padding: multiple of every k-chunk of g = a Omega
constexpr int kGemm2MaxSplits = 32;  // most row splits of one strip of a^T g
// Longest FP32 accumulation chains of the precision modes (FP32, BF16X2): rows of a per row-split
// partial of a^T g, columns per k split of g = a Omega.
constexpr int64_t kPrecRows = 512, kPrecCols = 4096;
// Fills the launch parameters of `it` (nrows, n, A, lda and the pointers set) for a P1 capacity of
// `splits_max` partials.
void plan_item(PassItem& it, int mode, int src, int splits_max);
// Assigns the first-workgroup offsets of `count` planned items and the group's grid sizes.
void plan_group(PassGroup& g, PassItem* items, int count);
// Strips of a^T g for n columns in `mode` (sizes the row-split scratch and counters).
int64_t gemm2_strips(int64_t n, int mode);
int64_t gemm2_strip_width(int mode);
// Most (strip, row split) partial tiles of a^T g one item can have (sizes the partial scratch).
int64_t gemm2_partial_tiles_max();
// Bound on (strip, row split) partial tiles of one item of at most `rows` rows and n columns.
int64_t gemm2_partial_tiles_bound(int64_t n, int64_t rows, int mode);
hipError_t launch_gemm1(const PassGroup& g, hipStream_t s);
hipError_t launch_reduce1(const PassGroup& g, hipStream_t s);
// a^T g, plus (for items split over rows) the fixed-order sum of the row-split partials into H
hipError_t launch_gemm2(const PassGroup& g, hipStream_t s);
// FP8 mode: amax of the block, then a' = e4m3(a 2^e) into `q` (nrows x ldq bytes).
// A block whose amax is not finite sets *nonfinite (and *nf_host when not null).
hipError_t launch_fp8_quantize(const float* A, int64_t lda, int nrows, int64_t n, uint32_t* amax,
                               uint8_t* q, int64_t ldq, int* exp_out, int* nonfinite, int* nf_host,
                               hipStream_t s);

// ---------------------------------------------------------------- small helpers
hipError_t launch_fill_f64(double* p, int64_t count, double v, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s);
// rows x cols block of a row-major matrix with leading dimension ld
hipError_t launch_fill_rows(double* p, int64_t rows, int cols, int64_t ld, double v,
                            hipStream_t s);
hipError_t launch_copy_state(int mode, const void* G, int64_t ldg, int64_t rows, const double* H,
                             int64_t ldh, int64_t n, int l, double* Gout, double* Hout,
                             hipStream_t s);
hipError_t launch_scale_f64(double* p, int64_t count, double a, hipStream_t s);
// a(:, 0:cols) += b(:, 0:cols) over `rows` rows (column-major FP64)
hipError_t launch_add_cols(double* a, int64_t lda, const double* b, int64_t ldb, int64_t rows,
                           int cols, hipStream_t s);
// *diff += number of entries whose bit patterns differ (column-major FP64; *diff zeroed by caller)
hipError_t launch_count_diff(const double* a, int64_t lda, const double* b, int64_t ldb,
                             int64_t rows, int cols, unsigned* diff, hipStream_t s);
hipError_t launch_copy_omega_out(const double* om64, int64_t ldo, int64_t n, int l, double* out,
                                 int64_t ld, hipStream_t s);

// ---------------------------------------------------------------- finalize (Alg. 4 steps 9-19)
// The finalize's small read-backs to the host (acceptance flags, the rank): with a pinned host
// buffer of kHostPinBytes and an event, a read-back copies into the buffer and waits by polling
// the event, which returns within microseconds of the copy; with either missing it copies into
// the destination and synchronises the stream.  bytes = 0 only waits for the stream's work.
constexpr size_t kHostPinBytes = 4096;
hipError_t read_back(void* dst, const void* src, size_t bytes, hipStream_t s, void* pin,
                     hipEvent_t ev);
// As read_back, for two device ranges at once (one wait): src1 to dst1 and src2 to dst2.
hipError_t read_back2(void* dst1, const void* src1, size_t bytes1, void* dst2, const void* src2,
                      size_t bytes2, hipStream_t s, void* pin, hipEvent_t ev);

struct FinalizeArgs {
  int mode;
  int64_t m, n;
  int k, l, b, LP;
  const void* G; int64_t ldg;        // m-side, column-major
  const double* H; int64_t ldh;      // n-side, column-major
  const double* om64; int64_t ldo;   // Omega' (FP64), n-side
  double* Q; int64_t ldq;            // m x l basis
  double* Q2 = nullptr;              // second m x l FP64 matrix (ld ldq) for b = l, or null
  double* Bt; double* Qb; int64_t ldb;   // B^T and the Q factor of B^T, n-side
  double* tsqr_ws; int64_t tsqr_ws_elems;
  double* red_ws; int64_t red_ws_elems;
  double* small;                     // small matrices, see finalize.hip
  Ctrl* ctrl;
  double* S; double* U; int64_t ldu; double* V; int64_t ldv;
  int32_t centre = 0;                // 1: column l of H holds s_A = A^T 1; centre G and H first
  double* mu = nullptr;              // out (centre): the column means, n values
  int32_t force_loop = 0;            // in: 1 takes the Householder TSQR path of the loop directly
  int32_t force_rb = 0;              // in: 1 Gram-Schmidt + TSQR for R_B, 2 shifted Cholesky QR3,
                                     //     3 QR2 formed, then treated as not accepted,
                                     //     4 as 3 with QR2's first pivot failing
  int32_t path_loop = -1;            // out: 0 Cholesky QR of the blocks, 1 Householder TSQR,
                                     //      2 one block (b = l) by Cholesky QR2
  int32_t path_rb = -1;              // out: 0 Cholesky QR2 of B^T, 2 shifted Cholesky QR3,
                                     //      1 Gram-Schmidt + TSQR
  void* host_pin = nullptr;          // pinned host staging of the read-backs (kHostPinBytes), or null
  hipEvent_t host_ev = nullptr;      // event the read-backs poll, or null
  Ctrl* ctrl_host = nullptr;         // out, if not null: the control block, read with the last
  bool ctrl_read = false;            //   wait when no device work followed it (ctrl_read set)
};
// Power scheme with P = 1: Omega_2 = sqrt(n) orth(H) (FP64, column-major) for the second pass.
struct PowerArgs {
  int64_t n;
  int l, b;
  const double* H; int64_t ldh;      // n x l, column-major
  double* om64; int64_t ldo;         // out: n x l (the padding is left as it is)
  double* W1; double* W2; int64_t ldw;   // two n x l scratch matrices
  double* red_ws; double* tsqr_ws; double* small;
  int32_t route = 0;                 // in: 0 Cholesky QR2, then shifted QR3, then TSQR as needed;
                                     //     2 shifted QR3 first; 1 Gram-Schmidt + TSQR
  int32_t route_used = -1;           // out: the route that produced orth(H)
  void* host_pin = nullptr;          // as in FinalizeArgs
  hipEvent_t host_ev = nullptr;
};
hipError_t run_power_omega(PowerArgs& p, hipStream_t s);
// Implicit centring of the sketch in place: G <- G - 1 (Omega'^T mu)^T, H <- H - mu (G^T 1)^T with
// mu = H(:, l) / m (column l of H holds A^T 1); writes mu (n values).
hipError_t centre_sketch(int mode, void* G, int64_t ldg, int64_t m, double* H, int64_t ldh,
                         int64_t n, int l, const double* om64, int64_t ldo, double* mu,
                         double* small, int b, hipStream_t s);
constexpr int kMaxDevices = 64;
// Once per device and thread-safe: kernel attributes the finalize needs (call on the device used).
hipError_t finalize_prepare();
// The pair table of one Jacobi sweep over n columns (host memory); rounds, or -1 (finalize.hip).
int jacobi_schedule(int n, uint8_t* out, int64_t cap);
size_t finalize_small_elems(int l, int b);
size_t tsqr_workspace_elems(int64_t rows, int b);
size_t reduce_workspace_elems(int64_t rows, int p, int q);
hipError_t run_finalize(FinalizeArgs& f, hipStream_t s);

}  // namespace sk
