// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modp.hpp"

namespace snc {

constexpr int KMAX = 3072;        // primes in the modulus table (log2 of their product ~ 92100)
constexpr int LPS = 2884;         // limb stride of the prime-product table (30*3072/32 + 4)
constexpr int MAXY_FAST = 64;     // largest y-degree handled by the register-resident elimination
constexpr int MAXY_GEN = 255;     // largest y-degree handled at all
constexpr int EE_WAVES = 1;       // wavefronts per eval_elim workgroup
constexpr int EE_BLOCK = 64 * EE_WAVES;
constexpr int INTERP_THREADS = 1024;
constexpr int MAX_D = 10000;     // largest degree bound: interpolation keeps 4(D+1)+O(1) words in LDS
constexpr int CRT_COEF_PER_BLOCK = 4;   // one wavefront per coefficient (digits)
constexpr int CRT_COMB_PER_BLOCK = 2;   // coefficients per combination workgroup (four wavefronts over limbs)
constexpr int GCD_THREADS = 256;

// One resultant res_y(f, g).  A is the operand of larger y-degree (m >= n);
// rows of A and B are listed top-down (row m of A first) so that the
// register arrays of the elimination are "top-aligned".
struct ResJob {
  int32_t m, n;        // y-degrees of A and B over Z[x], m >= 1, m >= n >= 0
  int32_t sign;        // 1: operands were swapped and m*n is odd (result negated)
  int32_t D;           // evaluation points x_j = j, j = 0..D
  int32_t k;           // primes 0..k-1 of the table
  int32_t T;           // residues per prime (coefficients of f and g)
  int32_t L;           // output limbs per coefficient
  int32_t nl;          // limbs per input coefficient
  int32_t rows_off;    // first RowDesc of A (rstride groups), then those of B
  int32_t rstride;     // row groups per operand: ceil((width + 1) / 4), width = register class or m
  int64_t coef_off;    // input limbs, limb-major [nl][T] (uint32 index)
  int64_t res_off;     // residues [k][T] (uint32 index)
  int64_t val_off;     // coefficients mod p: [k][D+1]
  int64_t pts_off;     // values at the points: [k][D+1]
  int64_t nq_off;      // Newton blocks Q_j of the block-parallel interpolation: [k][64 ceil((D+1)/64)]
  int64_t dig_off;     // mixed-radix digits [D+1][k]
  int64_t acc_off;     // CRT accumulator [D+1][LX] with LX = lx_of(k)
  int64_t out_off;     // output limbs [D+1][L]
};

// Rows of an operand are stored top-down (row of y^deg first) in groups of
// four: group g holds rows 4g..4g+3 interleaved coefficient-major, zero-padded
// to the longest of the four: residue off + 4c + q = coefficient of x^c of row
// 4g + q.
struct RowDesc {
  int32_t off;  // first residue of the group within a prime's block of T
  int32_t len;  // coefficients per row of the group (0 for an all-zero group)
};
// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin by
// block index.  Renumbering so that XCD x runs a contiguous range of logical
// blocks keeps neighbouring work, which reads the same data (the residues of
// one prime, adjacent coefficients), in one L2.  A bijection on [0, nb).
constexpr int NXCD = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t q = nb / NXCD, r = nb % NXCD, x = b % NXCD;
  return x * q + (x < r ? x : r) + b / NXCD;
}

constexpr int ROWGRP = 4;
constexpr int HCHUNK = 4;   // Horner steps per 64-byte scalar load; group lengths are padded to a multiple
__host__ __device__ inline int padded_group_len(int ml) { return (ml + HCHUNK - 1) / HCHUNK * HCHUNK; }

// Constant tables of a Chinese-remainder reconstruction over primes
// q_0..q_{k-1}: garner[i] = Montgomery form of (Q_i mod q_i)^-1 and
// wtab[j*wstride + i] = Montgomery form of Q_j mod q_i with Q_j = prod_{l<j} q_l;
// ptab row j (pstride limbs) = Q_j.
struct CrtTables {
  const PrimeC* primes;
  const uint32_t* garner;
  const uint32_t* wtab;
  const uint32_t* ptab;
  int32_t wstride, pstride;
};

// One gcd problem in Z[x]: a and b of degrees da, db >= 1; its primes are
// "slots" (table index per slot), filled in rounds of nslots starting at slot0.
struct GcdDesc {
  int32_t da, db;          // degrees of a and b
  int32_t nl;              // limbs per input coefficient
  int32_t wl;              // row length of w: min(da, db) + 1
  int32_t deriv;           // 1: b = a' (only a's limbs are stored; b's residues are formed from them)
  int32_t fused;           // 1: a's residues are given (plain, vals[slot * vstride + i]), b = a'; only
                           //    e and the degree of a mod p are written
  const uint32_t* vals;    // fused: residues of a, coefficient i of slot s at vals[s * vstride + i]
  int64_t vstride;
  int64_t d_off;           // fused: int32 per slot, degree of a mod p
  int64_t coef_off;        // input limbs [(da+1)+(db+1)][nl], or [da+1][nl] when deriv (uint32 index)
  int64_t slot_prime_off;  // int32 per slot: index of its prime in the modulus table
  int64_t res_off;         // residues [slot][da+db+2] (Montgomery)
  int64_t e_off;           // int32 per slot: degree of the gcd mod p, -2 if p divides both leading coefficients
  int64_t w_off;           // [slot][wl]   monic gcd mod p (plain)
  int64_t u_off;           // [slot][da+1] a / monic gcd mod p (plain)
  int64_t v_off;           // [slot][db+1] b / monic gcd mod p (plain)
  int32_t* ed_out;         // fused: if set, e and d are written at ed_out + e_off / d_off (host-mapped)
};

// gcd degree written for a prime dividing both leading coefficients (the prime is not used)
constexpr int32_t GCD_SLOT_UNUSABLE = -2;

// abnormal (prime, point) instance queued for the general elimination
struct AbnEntry {
  int32_t job, prime, point, pad;
};
// value left at an abnormal instance's point until the general pass (no residue is >= 2^30)
constexpr uint32_t ABN_MARK = 0xffffffffu;
// capacity of the abnormal-instance list of a batch of ninst instances
inline uint32_t abn_list_cap(int64_t ninst) {
  const int64_t c = ninst / 16 > 4096 ? ninst / 16 : 4096;
  return (uint32_t)(c < ninst ? c : ninst);
}

__host__ __device__ inline int lx_of(int k) { return (30 * k + 31) / 32 + 2; }

// launchers (kernels_res.hip)
void upload_tables(const PrimeC* primes, const uint32_t* garner_c, const uint32_t* wtab,
                   const uint32_t* ptab, hipStream_t s);
hipError_t configure_kernels();
void launch_ifact_init(hipStream_t s);
size_t interp_lds_bytes(int max_D);
// block-parallel interpolation: one workgroup per (resultant, prime, block of 64 coefficients),
// for degree bounds below 64 IFF_J and the first IFF_K primes (falling-factorial table)
constexpr int IFF_J = 16;
constexpr int IFF_K = 256;
inline bool interp_blk_fits(int max_D, int max_k) { return max_D + 1 <= 64 * IFF_J && max_k <= IFF_K; }
void launch_interp_blk(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks, uint32_t* ws,
                       uint32_t* zero_word, hipStream_t s);
void launch_zero_u32(uint32_t* p, int64_t n, hipStream_t s);
// one-wavefront interpolation per (resultant, prime): degree bounds up to IW_MAXD, for batches with at
// least IW_MIN_PAIRS (resultant, prime) pairs; jobs from job_list_d (prefix: k per job)
constexpr int IW_MAXD = 4095;
constexpr int64_t IW_MIN_PAIRS = 4096;
void launch_interp_w(const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d, int njobs,
                     int64_t nblocks, int max_D, uint32_t* ws, uint32_t* zero_word, hipStream_t s);
// zero_word (may be null) is set to zero by the same launch
void launch_reduce(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                   const uint32_t* ws, uint32_t* res_base, uint32_t* zero_word, hipStream_t s);
// the evaluation kernel stages a prime's residues in LDS up to this size
constexpr int EE_LDS_MAX = 64 * 1024;
inline bool eval_elim_in_lds(int max_T) { return (size_t)max_T * sizeof(uint32_t) <= (size_t)EE_LDS_MAX; }
// Launch variant of the evaluation kernel for one register class:
//   wpe: minimum wavefronts per SIMD the register allocation is held to (1..4, 1 = unconstrained);
//   chunk: 0 = one workgroup per block; > 0 = persistent grid of `grid` workgroups taking `chunk`
//          blocks at a time from a counter that is zero at launch.
struct EEVariant {
  int32_t wpe = 1;
  int32_t chunk = 0;
  int64_t grid = 0;
};
constexpr int EE_WPE_MAX = 4;
// Revision of the evaluation kernels' code and of the tuner's choice rule,
// part of the autotuner's cache file name: a changed kernel is tuned again
// instead of taking stale choices.
constexpr int EE_KERNEL_REV = 5;
// workgroups of a variant resident on the whole device (0 if the query fails)
int eval_elim_grid(int cls, int wpe, int max_T);
// private (spill) bytes per lane of a variant's kernel (-1 if the query fails)
int eval_elim_scratch(int cls, int wpe, int max_T);
// reduce_in: the residues are reduced from the input limbs inside the kernel (LDS variant only)
void launch_eval_elim(int cls, const EEVariant& v, uint32_t* counter, const ResJob* jobs_d,
                      const int32_t* job_list_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                      int max_T, const RowDesc* rows_d, uint32_t* ws, uint32_t* abn_count, AbnEntry* abn_list,
                      uint32_t abn_cap, bool reduce_in, hipStream_t s);
// abnormal instances: the list when count <= cap, else a scan of every
// instance for ABN_MARK (inst_prefix: prefix sums of k (D+1) over the jobs)
void launch_elim_general(const ResJob* jobs_d, const RowDesc* rows_d, uint32_t* ws,
                         const uint32_t* abn_count, const AbnEntry* abn_list, uint32_t cap,
                         const int64_t* inst_prefix_d, int njobs, hipStream_t s);
void launch_elim_general_all(const ResJob* jobs_d, const int32_t* job_list_d,
                             const int64_t* inst_prefix_d, int njobs, int64_t ninst,
                             const RowDesc* rows_d, uint32_t* ws, hipStream_t s);
// the interpolation launches also clear zero_word (the abnormal-instance counter)
void launch_interp(const ResJob* jobs_d, const int64_t* blk_prefix_d, int njobs, int64_t nblocks,
                   int max_D, uint32_t* ws, uint32_t* zero_word, hipStream_t s);
// job_list_d: the jobs of the launch (block prefix over them), or null for jobs 0..njobs-1
void launch_crt_digits(const CrtTables& tb, const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d,
                       int njobs, int64_t nblocks, uint32_t* ws, hipStream_t s);
void launch_crt_combine(const CrtTables& tb, const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d,
                        int njobs, int64_t nblocks, int kmax, uint32_t* ws, hipStream_t s);
// Chinese remaindering of a resultant with at most CRT_SMALL_K[cls] primes of
// the modulus table: one lane per coefficient (digits and binary value in one
// kernel); blocks of 64 coefficients, prefix over the launch's jobs
constexpr int NCRT_SMALL = 3;
constexpr int64_t CRT_SMALL_MIN_COEFS = 64 * 256;  // a wavefront per CU
constexpr int CRT_SMALL_K[NCRT_SMALL] = {32, 64, 128};
inline int crt_small_class(int k) {
  for (int c = 0; c < NCRT_SMALL; ++c)
    if (k <= CRT_SMALL_K[c]) return c;
  return -1;
}
void launch_crt_small(int cls, const ResJob* jobs_d, const int32_t* job_list_d, const int64_t* prefix_d, int njobs,
                      int64_t nblocks, uint32_t* ws, hipStream_t s);
void launch_crt_small_init(hipStream_t s);  // transposed table of P_j mod p_i (once per device)
CrtTables global_crt_tables();  // the resident tables of the modulus table (after upload)

// gcd work items are (problem, slot) pairs indexing a device array of GcdDesc
void launch_gcd_reduce(const GcdDesc* descs, const int32_t* items, int nitems, int max_rows, int max_nl,
                       uint32_t* ws, hipStream_t s);   // residues of a, b per item (rows: stored coefficient rows)
int gcd_reg_slots(int maxd);             // register class of a degree (slots per lane), 0: LDS kernel
constexpr int GCD_MAX_DEG = 13000;       // the LDS kernel keeps 3 (deg + 1) words
void launch_gcd_euclid(const GcdDesc* descs, const int32_t* items, int nitems, int slots, int maxd, uint32_t* ws,
                       hipStream_t s);   // monic gcd and cofactors per item; one register class per launch
// selected slots sel_d[j] (primes sprimes_d[j]) into compact rows; scales_d[3j..3j+2] = beta,
// cont(a)^-1, cont(b)^-1 mod q_j (plain) multiply w, u, v
void launch_gcd_gather(const GcdDesc& G, const int32_t* sel_d, const uint32_t* scales_d, const PrimeC* sprimes_d,
                       int ks, int e, uint32_t* ws, int64_t wv, int64_t uv, int64_t vv, hipStream_t s);
hipError_t configure_gcd_kernels();
// blocked Euclid of the square-free check (a workgroup of eight wavefronts per
// (problem, prime), fused descriptors only) for the register classes 6, 9, 12, 16
bool gcd_lehmer_class(int slots);
size_t gcd_lehmer_lds_bytes(int slots);
void launch_gcd_lehmer(const GcdDesc* descs, const int32_t* items, int nitems, int slots, uint32_t* ws,
                       hipStream_t s);

// Per-(prime, point) images of a bivariate gcd (k_ygcd): A and B (rows in y
// of polynomials in x, dense rectangles of residues) evaluated at
// x_j = j + shift, W_j = gamma(x_j) * monic gcd_y(A(x_j, y), B(x_j, y)) mod p.
struct YGcdArgs {
  const PrimeC* primes;
  const uint32_t* res;   // Montgomery residues [k][T]
  int32_t T, k, npts;    // residues per prime, primes, points
  int32_t mA, dxA, offA; // A: row i, coefficient of x^t at offA + i (dxA + 1) + t
  int32_t mB, dxB, offB;
  int32_t offG, dg;      // gamma: coefficient of x^t at offG + t, degree dg
  int32_t emax;          // coefficients 0..emax of W are written
  int32_t cap;           // LDS columns hold cap + 1 words (cap >= mA, mB)
  uint32_t shift;
  int32_t* e_out;        // [k][npts]: degree of the gcd, -1 at a point where a leading coefficient vanishes
  uint32_t* w;           // coefficient i of W at w[w_off + i w_stride + pi npts + j] (Montgomery)
  int64_t w_off, w_stride;
};
size_t ygcd_lds_bytes(int cap);
hipError_t configure_ygcd_kernel();
void launch_ygcd(const YGcdArgs& a, hipStream_t s);

int fast_class_of(int maxy);  // index of the register class for a y-degree, -1 if none
int fast_class_cap(int cls);

}  // namespace snc
