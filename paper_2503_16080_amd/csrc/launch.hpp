// launch.hpp -- host-side launchers of the libhlb kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace hlb {

// Tile shape of an INT8 GEMM instantiation: digits of each operand and workgroup tile.
struct I8Shape {
    int dp, dx;  // 0 when no instantiation exists
    int bm, bn;
};
// cls: tile class (0 = 128 x 64 outputs, 1 = 64 x 128 outputs) where the digits allow both.
I8Shape i8_shape(int dp, int dx, int cls);

// Digit split of the left operand (rows of P) into the tile-major workspace.
hipError_t launch_split_rows_i8(int D, int R, const int64_t *P, int64_t ldp, int64_t m, int64_t k,
                                int tiles, int kblocks, int8_t *out, hipStream_t s);
// Digit split of the right operand (columns of X, transposed) into the workspace.
hipError_t launch_split_cols_i8(int D, int R, const uint64_t *X, int64_t ldx, int64_t k, int64_t n,
                                int tiles, int kblocks, int8_t *out, hipStream_t s);
hipError_t launch_gemm_i8(int dp, int dx, int cls, const GemmArgs &a, hipStream_t s);
// Same tile with the digit products of shifts below `drop` (1..3) skipped; no K fold.
hipError_t launch_gemm_i8_trunc(int dp, int dx, int cls, int drop, const GemmArgs &a, hipStream_t s);
// Batch path: all splits of a batch in one launch, the work counter reset, and the
// persistent GEMM over every tile of every problem.
hipError_t launch_split_batch_i8(int D, const SplitJob *jobs, const int32_t *wg_job, int64_t total_wgs,
                                 hipStream_t s);
hipError_t launch_reset_counter(unsigned int *counter, hipStream_t s);
hipError_t launch_gemm_i8_batch(int dp, int dx, bool fold, const BatchArgs &a, int grid, hipStream_t s);

// FP64 form: limb counts of each operand; returns false when no instantiation exists.
bool f64_supported(int np, int nx);
// Register-staged kernel (any limb counts f64_supported accepts; no workspace).
hipError_t launch_gemm_f64(int np, int nx, const GemmArgs &a, hipStream_t s);
// One FP64 product of the rounded operands (plaintext signed, residues centred), reduced mod q.
hipError_t launch_gemm_f64_trunc(const GemmArgs &a, hipStream_t s);
// Plane path for one plaintext limb: preparation into double planes, then the direct-to-LDS
// GEMM (nx = 3 or 4 limbs; or nx = 1 with trunc, Strategy 2).  Workspace bytes per operand:
int64_t f64_plane_bytes_p(int64_t tiles_m, int64_t kblocks);
int64_t f64_plane_bytes_x(int nx, int64_t tiles_n, int64_t kblocks);
hipError_t launch_prep_p_planes(const int64_t *P, int64_t ldp, int64_t m, int64_t k, int tiles, int kblocks,
                                double *out, hipStream_t s);
hipError_t launch_prep_x_planes(int nx, bool trunc, const uint64_t *X, int64_t ldx, int64_t k, int64_t n, int tiles,
                                int kblocks, int w, uint64_t q, double *out, hipStream_t s);
hipError_t launch_gemm_f64_planes(int nx, bool trunc, const GemmArgs &a, hipStream_t s);

// Multimodular (CRT) INT8 form: residue splits (qc = 0: signed values; else residues mod qc
// taken centred; the left operand's residues are multiplied by scale.s[i] mod p_i), one INT8
// GEMM per modulus, recombination.  D must be crt_supported_d.
bool crt_supported_d(int D);
int crt_round_d(int D);  // smallest supported D >= D, or 0
struct CrtScale;
struct CrtGemmArgs;
struct CrtCombineArgs;
// variant 0: 256 x 128 output tiles; 1: 256 x 256 (both 8 waves).  crt_tile_cols gives the
// tile width.
int crt_tile_cols(int variant);
hipError_t launch_crt_gemm(int variant, const CrtGemmArgs &a, int workers, hipStream_t s);
// Batched forms: one launch for many operands (jobs in increasing wg_start), one GEMM launch
// per tile class for many problems (256 x crt_tile_cols(variant) tiles), one launch for many
// recombinations (crt_combine_wgs workgroups each).
struct CrtSplitJob;
struct CrtBatchArgs;
struct CrtCombineJob;
hipError_t launch_crt_split_batch(int D, const CrtSplitJob *jobs, int njobs, int64_t total_wgs, const CrtScale &scale,
                                  hipStream_t s);
// persistent: `workers` workgroups (at most one per CU fits), counters zeroed beforehand
hipError_t launch_crt_gemm_batch(int variant, const CrtBatchArgs &a, int workers, hipStream_t s);
int64_t crt_combine_wgs(int64_t m, int64_t n);
hipError_t launch_crt_combine_batch(const CrtCombineJob *jobs, int njobs, int64_t total_wgs, hipStream_t s);
// The same two with the job tables in the kernel arguments (at most kCrtTabSplit operands /
// kCrtTabCombine outputs per launch).
struct CrtSplitTable;
struct CrtCombineTable;
hipError_t launch_crt_split_tab(int D, const CrtSplitTable &t, int64_t total_wgs, const CrtScale &scale,
                                hipStream_t s);
hipError_t launch_crt_combine_tab(const CrtCombineTable &t, int64_t total_wgs, hipStream_t s);

// Auxiliary kernels.
hipError_t launch_validate(const uint64_t *X, int64_t rows, int64_t cols, int64_t ld, uint64_t q,
                           unsigned long long *first_bad, hipStream_t s);
hipError_t launch_absmax(const int64_t *P, int64_t m, int64_t k, int64_t ld,
                         unsigned long long *out, hipStream_t s);
// `value` (launch_fill) or zeros (launch_zero) in a rows x cols block of 64-bit words with row
// stride ld.
hipError_t launch_fill(uint64_t *C, int64_t rows, int64_t cols, int64_t ld, uint64_t value, hipStream_t s);
hipError_t launch_zero(uint64_t *C, int64_t rows, int64_t cols, int64_t ld, hipStream_t s);
hipError_t launch_encode(const double *M, int64_t count, double delta, int64_t *out, hipStream_t s);
// D[i] = (sign * AS[i] + E[i]) mod q elementwise over `count` entries, with AS residues and
// E signed: used by the test-only encrypt (sign = -1) and decrypt (sign = +1, E = residues).
hipError_t launch_combine(const uint64_t *AS, const int64_t *Es, const uint64_t *Eu, int sign,
                          int64_t count, uint64_t q, uint64_t *out, hipStream_t s);
hipError_t launch_rescale(const uint64_t *X, int64_t count, const RescaleConsts &rc, uint64_t *Y, hipStream_t s);
hipError_t launch_residues_of_signed(const int64_t *v, int64_t count, uint64_t q, uint64_t *out,
                                     hipStream_t s);

}  // namespace hlb
