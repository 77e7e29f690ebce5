// Internal declarations shared by the runtime and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zippir.h"

namespace zp {

// Native 16-byte vector (usable with the nontemporal load builtin).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Per-client constants, all device pointers into one allocation.
//   N2  S limbs   N^2 (zero padded)          R1  S limbs   R mod N^2, R = 2^(32 S)
//   RR  S limbs   R^2 mod N^2                NP  S limbs   N (zero padded, S-limb layout)
//   Nn  SN limbs  N                          C1  SN limbs  R_N mod N, R_N = 2^(32 SN)
//   C2  SN limbs  R_N^2 mod N              CP  S limbs   2^(64 S - 32) mod N^2 (K' -> K R)
//   D1  SN limbs  R_N^2 2^-32 mod N         D2  SN limbs  R_N^3 2^-32 mod N
//   (D1, D2 map K' = lo + hi R_N to (K mod N) R_N mod N with two Montgomery products)
//   C96 SN limbs  2^96 R_N mod N (x -> x 2^96 mod N in one Montgomery product)
//   CT  SN limbs  2^t R_N mod N (x -> x 2^t mod N, t the packing shift; unused by the kernels
//                 since the packed offset answer takes per-row powers PJ)
struct ClientDev {
  const uint32_t* N2;
  const uint32_t* R1;
  const uint32_t* RR;
  const uint32_t* NP;
  const uint32_t* Nn;
  const uint32_t* C1;
  const uint32_t* C2;
  const uint32_t* CP;
  const uint32_t* D1;
  const uint32_t* D2;
  const uint32_t* C96;
  const uint32_t* CT;
  uint32_t m2prime;  // -(N^2)^{-1} mod 2^32
  uint32_t nprime;   // -N^{-1} mod 2^32
  int L;             // limbs of a ciphertext (2h)
  int h;             // limbs of N
  int P;             // limbs per lane for mod-N^2 numbers (S = 64 P >= L)
  int PN;            // limbs per lane for mod-N numbers (SN = 64 PN >= h)
};

// Online kernels stream at most this many bytes of D per launch (larger databases are cut
// into row chunks), bounding how long one database's launch holds the device.
constexpr long long kLaunchBytes = 2LL << 30;

// 8-bit fixed-base windows: the standalone compressor's table, and the client hint's for
// few rows.
constexpr int kWindowBits = 8;
constexpr int kWindows = 32 / kWindowBits;
constexpr int kDigits = (1 << kWindowBits) - 1;

// ---- matvec.hip
// planes: 4 consecutive byte arrays of `pitch` bytes, plane b holding byte b of every
// query entry (zero beyond cols).  One query.  Also clears b (rows entries), which
// launch_matvec accumulates into.
void launch_pack_planes_u8(const uint32_t* q, int cols, int pitch, uint8_t* planes, uint32_t* b,
                           int rows, hipStream_t s);
void launch_matvec(const uint8_t* D, int rows, int pitch, const uint8_t* planes, uint32_t* b,
                   hipStream_t s);

// ---- answer.hip
// Column segments of the two-launch step (at most 64: one partial per lane of the combine).
int answer_segments(int pitch);
// part[j * nseg + s] = row j of D times query q (cols uint32, 16-byte aligned) over column
// segment s, mod 2^32, for the nseg = answer_segments(pitch) segments; no packing of q and no
// clearing needed.
void launch_matvec_part(const uint8_t* D, int rows, int pitch, const uint32_t* q, int cols,
                        uint32_t* part, hipStream_t s);
// b_j = sum_s part[j * nseg + s] mod 2^32 (nseg <= 64) and C = K (1 + b N) mod N^2 (rows x L),
// from K' and M' as launch_compress takes them.
void launch_combine_parts(const ClientDev& cd, const uint32_t* Kp, const uint32_t* Mp,
                          const uint32_t* part, int nseg, int rows, uint32_t* b, uint32_t* C,
                          hipStream_t s);

// ---- gemm_i8.hip
// Signed byte planes of `ncol` vectors: X element (c, i) is x[c*stride_c + i*stride_i].
// Xs[(c*4 + b)*pitch + i] = (byte b of X(c,i)) ^ 0x80 for i < cols, 0 beyond.
// colsum[c*4 + b] = sum_{i<cols} Xs[(c*4+b)*pitch + i].
void launch_pack_planes_s8(const uint32_t* x, long long stride_c, long long stride_i, int ncol,
                           int cols, int pitch, int8_t* Xs, int32_t* colsum, hipStream_t s);
// rowsum[j] = sum_{i<cols} (D[j][i] - 128)
void launch_rowsum(const uint8_t* D, int rows, int cols, int pitch, int32_t* rowsum,
                   hipStream_t s);
// out = D . X mod 2^32 for `rows` rows of D starting at D, all ncol columns (out is
// overwritten).  out_rowmajor: out[j*ncol + c]; otherwise out[c*out_ld + j].
// Launch shape: `waves` per block, `depth` K steps of D in flight per wave, `mr` x 16 rows per
// wave, `kb` bytes of K per step, `ksplit` K ranges per output tile.  Every shape gives
// identical bits; gemm_shape_valid tells whether a shape is built and fits the pitch.
// cg (one plane only): 32-vector column groups per block, 2..4.
struct GemmShape {
  int waves, depth, mr, kb, ksplit, cg;
};
bool gemm_shape_valid(const GemmShape& sh, int pitch, int planes);
// planes = 4: X holds uint32 vectors as four byte planes (launch_pack_planes_s8) and
// out = D . X mod 2^32.  planes = 1: X holds uint8 vectors as one plane,
// Xs[c*pitch + i] = X(c,i) ^ 0x80 (0 beyond cols), colsum[c] = sum_{i<cols} Xs[c*pitch + i],
// and out = D . X, exact while cols * 255^2 < 2^32.
// tiled: D is the tiled copy of a row range starting at a multiple of 16 rows (four planes only)
void launch_gemm_planes(const uint8_t* D, int rows, int cols, int pitch, int planes,
                        const int8_t* Xs, const int32_t* colsum, int ncol, const int32_t* rowsum,
                        uint32_t* out, bool out_rowmajor, long long out_ld, const GemmShape& sh,
                        hipStream_t s, bool tiled = false);
// ---- hgemm.hip: H = D.A mod 2^32 (rows x n, row-major) on int8 MFMA
// A's signed byte planes in fragment order (layout in hgemm.hip): Apt holds 4 x hgemm_npad(n) x
// pitch bytes.  Acolsum[k 4 + b] = sum_{i<cols} (byte b of A[i][k]) - 128.
int hgemm_npad(int n);
void launch_a_planes(const uint32_t* A, int cols, int n, int pitch, uint8_t* Apt, hipStream_t s);
void launch_a_colsum(const uint32_t* A, int cols, int n, int32_t* Acolsum, hipStream_t s);
// D is the tiled copy (tiled) or row-major rows x pitch; rowsum as launch_rowsum.
// `variant` < hgemm_variants() picks the launch shape (identical bits for every one).
int hgemm_variants();
void launch_hgemm(const uint8_t* D, bool tiled, int rows, int cols, int pitch, const uint8_t* Apt, int n,
                  const int32_t* Acolsum, const int32_t* rowsum, uint32_t* H, int variant, hipStream_t s);

// ---- batch.hip: the fused, persistent batched answer on the tiled copy Dt
// B[c ldb + j] = D.Q[c] mod 2^32 for c < batch (Q batch x cols uint32, query c at Q + c cols),
// j < rows; rowsum as launch_rowsum.  Shapes: mr 16-row tiles per wavefront (1 or 2), depth
// K steps of D in flight (2..4), ksplit K ranges per row block (0: enough to fill num_cus),
// blocks_per_cu persistent workgroups per CU.  Every shape gives identical bits.
struct BatchShape {
  int mr, depth, ksplit, blocks_per_cu;
};
bool batch_answer_supported(int rows, int pitch);
void launch_batch_answer(const uint8_t* Dt, int rows, int cols, int pitch, const uint32_t* Q, int batch,
                         const int32_t* rowsum, uint32_t* B, long long ldb, const BatchShape& sh,
                         int num_cus, hipStream_t s);

// Tiled copy for the contraction: Dt[(j/16) 16 pitch + (i/64) 1024 + (j%16) 64 + i%64] = D[j pitch + i]
// for the listed rows (device list; nullptr: rows 0 .. nrows-1).
void launch_tile_rows(const uint8_t* D, int pitch, const uint32_t* rowlist, int nrows, uint8_t* Dt,
                      hipStream_t s);

// Tuning cross-check: with compare false, ref (rows x ncol, column c at ref + c*rows) receives
// a copy of the output block; with compare true, *mism is increased by the number of
// elements that differ from that copy.
void launch_gemm_snapshot(const uint32_t* out, int rows, int ncol, bool out_rowmajor,
                          long long out_ld, uint32_t* ref, bool compare, unsigned* mism,
                          hipStream_t s);

// ---- rows.hip (row gather/scatter for updates and partial recomputation)
void launch_gather_rows_u8(const uint8_t* src, int pitch, const uint32_t* rows, int nrows,
                           uint8_t* dst, hipStream_t s);
void launch_scatter_rows_u8(const uint8_t* src, int src_pitch, int cols, const uint32_t* rows,
                            int nrows, uint8_t* dst, int dst_pitch, hipStream_t s);
void launch_gather_rowsum(const int32_t* src, const uint32_t* rows, int nrows, int32_t* dst,
                          hipStream_t s);
void launch_scatter_rows_u32(const uint32_t* src, int width, const uint32_t* rows, int nrows,
                             uint32_t* dst, hipStream_t s);

// ---- hint.hip
// Fixed-base table of windows of wbits bits: entry (k, w, v) at table + ((k windows + w)
// (2^wbits - 1) + v - 1) S holds ck_k^(v 2^(wbits w)) R mod N^2, v = 1 .. 2^wbits - 1.
void launch_build_table(const ClientDev& cd, const uint32_t* ck, int n, int windows,
                        uint32_t* table, hipStream_t s, int wbits = kWindowBits);
// Rows processed: rowlist[i] for i < nrows (rowlist may be null: rows 0..nrows-1), with a
// table of ceil(32 / wbits) windows.  Writes K'_j = K_j 2^32 mod N^2 (rows x L limbs).
void launch_hint_rows(const ClientDev& cd, const uint32_t* H, int n, const uint32_t* rowlist,
                      int nrows, const uint32_t* table, int wbits, uint32_t* Kp, hipStream_t s);
// The same for few rows (hint_parts(nrows, n) > 1): each row's bases split into that many parts,
// one wavefront each, then joined; partial holds nrows x parts x 64P limbs.
constexpr int kSplitRowsBelow = 4096;
int hint_parts(int nrows, int n);
void launch_hint_rows_split(const ClientDev& cd, const uint32_t* H, int n, const uint32_t* rowlist,
                            int nrows, const uint32_t* table, int wbits, int parts, uint32_t* partial,
                            uint32_t* Kp, hipStream_t s);
// M'_j = N (K'_j mod N) (rows x L limbs), the combine key.
// (Y, when not NULL: rows x h, Y[row] = (K mod N) R_N mod N for the offset combine, where
// K = Kp 2^-32 when `scaled` and K = Kp otherwise.)
void launch_combine_key(const ClientDev& cd, const uint32_t* Kp, const uint32_t* rowlist,
                        int nrows, uint32_t* Mp, uint32_t* Y, hipStream_t s, bool scaled = true);
// K_j = K'_j 2^{-32} mod N^2 for rows [row0, row0+nrows) into K (nrows x L).
void launch_unscale(const ClientDev& cd, const uint32_t* Kp, int row0, int nrows, uint32_t* K,
                    hipStream_t s);

// ---- packed responses (batched compression, gamma = 2^t)
// Kg[g] = prod_{j} K_{g ell + j}^{2^(t j)} mod N^2 (canonical) for the listed groups, from K'.
void launch_group_keys(const ClientDev& cd, const uint32_t* Kp, int rows, int ell, int t,
                       const uint32_t* glist, int ngroups, uint32_t* Kg, hipStream_t s);
// x[i] <- x[i] 2^(32 limbs) mod N^2 for the listed rows of an L-limb array (2^(32 limbs) < N^2).
void launch_mul_pow2_limbs(const ClientDev& cd, uint32_t* x, const uint32_t* rowlist, int nrows,
                           int limbs, hipStream_t s);
// C[g] = K_g + beta_g M_g mod N^2 with beta_g = sum_j b[g ell + j] 2^(t j); Mr holds M_g 2^(32h).
void launch_compress_packed(const ClientDev& cd, const uint32_t* Kg, const uint32_t* Mr,
                            const uint32_t* b, int rows, int ell, int t, uint32_t* C, hipStream_t s);

// ---- offset answer of the full protocol (offset.hip)
// E planes of the contraction (layout in offset.hip): Ep holds rows_pad x 4 x 64 S bytes with
// S = offset_slices(n), rows_pad a multiple of 128; Ers (4 x rows_pad) receives the plane sums
// sum_{k<n} (byte a of E_jk) - 128 for rows below `rows` (the caller zeroes the rest once).
int offset_slices(int n);
void launch_e_planes(const uint32_t* H, int rows, int n, int rows_pad, uint8_t* Ep, int32_t* Ers,
                     hipStream_t s);
// Column tiles of 16 of the contraction: the 4h + 3 output positions, padded to whole column
// groups (offset.hip).
int offset_tiles(int h);
// out[k] = cko[k] 2^96 mod N (canonical) for the n offset entries of one client (h limbs each).
void launch_scale_offsets(const ClientDev& cd, const uint32_t* cko, int n, uint32_t* out,
                          hipStream_t s);
// The offset bytes of `batch` scaled offset vectors ys (batch x n x h limbs) in the
// contraction's staging order (offset.hip): Yf holds batch x offset_y_bytes(n, h) bytes; colsum
// (batch x 16 offset_tiles(h)) receives sum_{k<n} (byte c of ys[i][k]) - 128 for c < 4h.
long long offset_y_bytes(int n, int h);
void launch_pack_y(const uint32_t* ys, int batch, int n, int h, uint8_t* Yf, int32_t* colsum,
                   hipStream_t s);
// With W_pos = sum_k sum_a (byte a of E_jk) (byte pos - a of ys[i][k]) for pos < 4h + 3 (exact:
// below 4 n 255^2 < 2^32; zero beyond): X[j ldw + i cpc + l] = sum_{u<4} W_(4l+u) 2^(8u) for
// l <= h, every row j < rows and client i < batch (cpc >= h + 1 words per client).
// `variant` < offset_gemm_variants(h) picks the launch shape (identical bits for every one).
int offset_gemm_variants(int h);
void launch_offset_gemm(const uint8_t* Ep, const int32_t* Ers, int rows_pad, int rows, int n,
                        const uint8_t* Yf, const int32_t* colsum, int batch, int h, uint64_t* X,
                        long long ldw, int cpc, int variant, hipStream_t s);
// T[j] (h limbs) = (b[j] 2^96 + sum_l X[j*ldw + l] 2^(32 l)) 2^-96 mod N, l <= h, where X was
// computed from offsets scaled by 2^96 (launch_scale_offsets).  With part non-null (b unused),
// b[j] = sum_s part[j*nseg + s] mod 2^32 from launch_matvec_part, written to bout.
void launch_offset_reduce(const ClientDev& cd, const uint64_t* X, long long ldw, const uint32_t* b,
                          int rows, uint32_t* T, hipStream_t s, const uint32_t* part = nullptr, int nseg = 0,
                          uint32_t* bout = nullptr);

// C[j] = K_j (1 + T[j] N) mod N^2 for rows [0, rows): T is rows x h (any value below 2^(32h)),
// K_j from the stored K', Y[j] = (K_j mod N) R_N mod N (h limbs); C is rows x L.
// scaled = false: Kp holds K itself (canonical), as the packed group keys do.
void launch_compress_offset(const ClientDev& cd, const uint32_t* Kp, const uint32_t* Y,
                            const uint32_t* T, int rows, uint32_t* C, hipStream_t s,
                            bool scaled = true);
// Tg[g] = sum_j 2^(t j) T[g ell + j] mod N for the groups of ell rows (T rows x h, canonical);
// PJ holds 2^(t j) R_N mod N for j < ell (SN limbs each); Tmp is rows x h scratch.
void launch_offset_pack(const ClientDev& cd, const uint32_t* T, int rows, int ell,
                        const uint32_t* PJ, uint32_t* Tmp, uint32_t* Tg, hipStream_t s);

// ---- standalone LWE / RLWE compression (lwec.hip)
// Exponent source of one compressed ciphertext: LWE rows (A rows x n, B rows) or RLWE
// coefficients (A and B the ring elements' n coefficients, ks the coefficient indices).
// Entries are qw 32-bit words (little-endian), reduced modulo q in the kernel; q = 0 means 2^64.
struct LweBatch {
  const uint32_t* A;
  const uint32_t* B;
  const uint32_t* ks;  // NULL for LWE rows
  int rows, n, qw, windows;
  uint64_t q;
};
// parts > 1: each ciphertext's n bases are split over `parts` waves whose partial products
// (Montgomery form, S limbs each) go to Part (rows x parts); otherwise X gets the result.
// (rows x parts) work items; from kQuadItems items on, four items share a wavefront.
constexpr long long kQuadItems = 16384;
void launch_compress_lwe(const ClientDev& cd, const LweBatch& lb, const uint32_t* table, int parts,
                         uint32_t* Part, uint32_t* X, hipStream_t s);
// Multiplies groups of `fan` consecutive partial products (parts per row -> ceil(parts/fan));
// when one remains per row, multiplies in Enc(b; 1) = 1 + bN and writes X (rows x L).
void launch_reduce_parts(const ClientDev& cd, const LweBatch& lb, const uint32_t* Part, int parts,
                         int fan, uint32_t* Out, uint32_t* X, hipStream_t s);
// ck[k] = pck[k / t]^(2^(dbits (t - 1 - k mod t))) mod N^2 for k < n (unpacking of packed keys
// with delta = 2^dbits): one chain of squarings per packed ciphertext, each Montgomery product
// spread over a workgroup.  Residues are kept as unpack_digits(S) 7-bit digits, the Montgomery
// radix is R = 2^(7 unpack_digits(S)) > 4 N^2, and cdig (device) holds three digit arrays of
// that length: N^2, -(N^2)^{-1} mod R and R^2 mod N^2.
constexpr int unpack_digits(int S) { return 16 * (((32 * S + 2 + 6) / 7 + 15) / 16); }
void launch_unpack_chains(const ClientDev& cd, const uint8_t* cdig, const uint32_t* pck, int n, int t,
                          int dbits, uint32_t* ck, hipStream_t s);

// ---- prg.hip (random hint keys of the silent offline phase)
// The 32-byte seed as eight little-endian words: the ChaCha20 key (RFC 8439).
struct SeedKey {
  uint32_t w[8];
};
// out[(i n + k) L ...] = ck_r[k] of query first_query + i (i < count, k < n): the first
// ChaCha20 candidate below N^2 (N2: W words, the low bits(N^2) bits kept by top_mask on word
// W-1), zero-padded to L limbs.  Entries rejected kMaxAttempts times add one to *failures.
void launch_expand_key(const SeedKey& key, uint32_t first_query, int n, int count, const uint32_t* N2, int W,
                       uint32_t top_mask, int L, uint32_t* out, unsigned* failures, hipStream_t s);

// ---- runtime.cpp accessors used by the serving engine and the no-alloc entry point
hipStream_t server_stream(pir_server* s);
void server_shape(pir_server* s, uint32_t* rows, uint32_t* cols);
// pir_answer_compress's checks (client known and current, at most 64 column segments; nseg
// receives their number; the server's device made current) and its two launches on device
// arrays (dQ 16-byte aligned, part nseg x rows words), with no device allocation; `events`
// false skips the pir_profile events (whose creation allocates).
pir_status answer_compress_check(pir_server* s, uint32_t id, int* nseg);
pir_status answer_compress_launch(pir_server* s, uint32_t id, const uint32_t* dQ, uint32_t* dB, uint32_t* dC,
                                  uint32_t* part, bool events = true);
void set_error(const char* msg);  // sets the calling thread's pir_last_error() text
int server_device(pir_server* s);
// pir_answer on device arrays in steps, for a caller that interleaves other streams' work
// between them (the serving engine): answer_begin picks the path (*path PIR_PATH_AUTO on entry)
// and enqueues the query packing; answer_rows enqueues rows [r0, r0 + nr) of B (r0 a multiple
// of 256).  Both on the server's stream, which must be current.
pir_status answer_begin(pir_server* s, const uint32_t* dQ, uint32_t batch, uint32_t* dB, int32_t* path);
pir_status answer_rows(pir_server* s, const uint32_t* dQ, uint32_t batch, uint32_t* dB, int32_t path, uint32_t r0,
                       uint32_t nr);
// Attach the server to a serving engine (tunes and sizes the batched shapes for batches up to
// max_batch answered in steps of step_rows rows, then stops in-place tuning) or detach it.
pir_status server_serving(pir_server* s, bool on, uint32_t max_batch, uint32_t step_rows);

// ---- noalloc.hip: the static scratch array of pir_answer_compress_noalloc
// With `device` current: looks up that device's address of the array once (hipGetSymbolAddress)
// and returns it in *out (out may be NULL).
pir_status scratch_init(int device, uint32_t** out);
size_t scratch_words();

// ---- compress.hip
void launch_compress(const ClientDev& cd, const uint32_t* Kp, const uint32_t* Mp,
                     const uint32_t* b, int rows, uint32_t* C, hipStream_t s);

}  // namespace zp
