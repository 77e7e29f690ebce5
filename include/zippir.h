/*
 * zippir.h -- C ABI of the ZipPIR server hot path for AMD Instinct MI355X (gfx950).
 *
 * ZipPIR (Akhavan Mahdavi, Diaa, Kerschbaum) is SimplePIR-style LWE PIR whose per-row LWE
 * answer is compressed into a Paillier ciphertext.  The server side computes
 *
 *   global hint      H = D.A mod 2^32                       (Alg. 5 preamble; Sec. 4.3 "Reusability")
 *   exponents        E = (-H) mod 2^32                      (Alg. 2 multiplies by q - a; Alg. 4)
 *   client hint      K_j = prod_k ck_k^{E_jk} mod N^2       (Alg. 5 Hint = PaillierMatMul(H, ck))
 *   answer           b = D.qu mod 2^32                      (Alg. 5 Response, first line)
 *   compressed row   c_j = K_j * (1 + b_j N) mod N^2        (Sec. 4.3 "Smaller responses w/
 *                                                             Paillier addition": K (+) Enc(b; 1))
 *
 * Orientation: D is rows x cols uint8 (plaintext modulus p = 256), row-major.  A is
 * cols x n uint32, row-major.  A query has cols entries, an answer has rows entries.  The
 * paper writes the same protocol on the transpose of D (Alg. 5); a client here retrieves a
 * column of D.
 *
 * Big integers are little-endian arrays of uint32 limbs.  A client with an N_bits-bit
 * Paillier modulus N uses L = 2*ceil(N_bits/32) limbs per ciphertext (values in [0, N^2)).
 *
 * Conventions for every call:
 *   - Buffers named in a call are borrowed for that call only.  Data the server keeps
 *     (D, A, H, each client's ck and K) is copied into, or computed in, device memory the
 *     server owns and frees in pir_destroy / pir_remove_client.
 *   - ptr_flags says where the call's array arguments live: PIR_PTR_HOST (pageable or pinned
 *     host memory) or PIR_PTR_DEVICE (device memory on the server's device, e.g. a torch
 *     tensor's data pointer).  Row-index lists are always host arrays.
 *   - All device work is enqueued on the HIP stream given to pir_setup.  A call whose
 *     outputs are host buffers synchronizes that stream before returning; a call with
 *     device outputs returns once its work is enqueued (use pir_sync or the stream).
 *   - One pir_server must not be used from two threads at once.
 *   - No C++ exception crosses this interface.  On error the call returns a negative
 *     status, leaves the server usable, and pir_last_error() describes the failure.
 */
#ifndef ZIPPIR_H
#define ZIPPIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pir_server pir_server;
typedef int32_t pir_status;

#define PIR_OK        0
#define PIR_EINVAL   (-1)  /* bad argument: shape, size, parameter or unknown id            */
#define PIR_ENOMEM   (-2)  /* device or host allocation failed                               */
#define PIR_EDEVICE  (-3)  /* a HIP call failed; pir_last_error() has the HIP message        */
#define PIR_ESTALE   (-4)  /* a client hint is missing or out of date (call pir_hint)        */
#define PIR_EBUSY    (-5)  /* resource temporarily exhausted (serving admission)             */

#define PIR_PTR_HOST   0u
#define PIR_PTR_DEVICE 1u

/* Answer paths for pir_answer_path. */
#define PIR_PATH_AUTO   0  /* batch 1 -> PIR_PATH_MATVEC, batch > 1 -> PIR_PATH_MFMA               */
#define PIR_PATH_MATVEC 1  /* HBM-streaming u8 x u32 matvec, once per query                        */
#define PIR_PATH_MFMA   2  /* one fused int8-MFMA contraction over four byte planes of the batch   */

/*
 * Server side of Setup (Alg. 5): register the database and the public LWE matrix.
 *   out      receives the new server handle (NULL on failure).
 *   device   HIP device ordinal; hip_stream is a hipStream_t on that device (NULL = default).
 *   D        rows x cols uint8, row-major.   A  cols x n uint32, row-major.
 * 1 <= rows <= 2^30, 1 <= cols <= 2^24, 1 <= n <= 2^16.  The global hint H is computed
 * lazily by the first pir_hint.
 * Errors: PIR_EINVAL (zero or too large a size, NULL pointer; checked before any device
 * call), PIR_ENOMEM, PIR_EDEVICE.
 */
pir_status pir_setup(pir_server **out, int device, void *hip_stream,
                     const uint8_t *D, uint32_t rows, uint32_t cols,
                     const uint32_t *A, uint32_t n, uint32_t ptr_flags);

/* Frees every device buffer the server owns.  NULL is ignored. */
void pir_destroy(pir_server *srv);

/*
 * Register a client's public material (Alg. 5 Setup output sent to the server).
 *   N        ceil(N_bits/32) limbs of the Paillier modulus; odd, top bit at N_bits-1.
 *   ck       n ciphertexts of L = 2*ceil(N_bits/32) limbs each (ck[k] = Enc(s_k)), each < N^2.
 *   client_id receives the new id.
 * N_bits is in [64, 4096].  Theorem 1 (Sec. 3.1) requires N > q + n q^2 with q = 2^32 for the
 * compressed answer to decrypt correctly; smaller N is rejected with PIR_EINVAL.
 */
pir_status pir_add_client(pir_server *srv, const uint32_t *N, uint32_t N_bits,
                          const uint32_t *ck, uint32_t ptr_flags, uint32_t *client_id);

/*
 * Silent offline phase (Sec. 4.3, "Lowering offline communication costs" and "Supporting
 * multiple queries"): the client sends only N and a 32-byte seed, and the server expands the
 * seed into the random ciphertexts ck_r of Alg. 5's Setup, one n-vector per query, on the
 * device.  Registers `count` clients, one per query index first_query .. first_query+count-1,
 * each with its own key and hint (pir_hint, pir_offset_answer, pir_compress_offset, ...), and
 * writes their ids to client_ids (a host array of count entries).
 *   N, N_bits  as for pir_add_client (N read from host or device memory per ptr_flags).
 *   seed       32 bytes in host memory: the ChaCha20 key (RFC 8439).
 * Entry k of query q is uniform over [0, N^2): the ChaCha20 keystream under the 96-bit nonce
 * (q, k, r) (three little-endian words; r the attempt, from 0), read from block 0 on as
 * little-endian 32-bit words w_i, gives the candidate sum_i w_i 2^(32 i) over
 * ceil(bits(N^2)/32) words cut to bits(N^2) bits; the first candidate below N^2 is taken.
 * The client derives the same ck_r from the seed and decrypts it at query time.
 * count in [1, 4096].  Errors: PIR_EINVAL (as pir_add_client; count), PIR_ENOMEM,
 * PIR_EDEVICE (also if an entry is rejected 64 times in a row, probability below 2^-64).
 * On error no client is registered.
 */
pir_status pir_add_client_seeded(pir_server *srv, const uint32_t *N, uint32_t N_bits,
                                 const uint8_t *seed, uint32_t first_query, uint32_t count,
                                 uint32_t ptr_flags, uint32_t *client_ids);

/* Copy entries [k0, k0+nk) of a client's key ck (nk x L uint32): the uploaded ciphertexts, or
 * the ones expanded from a seed.  PIR_EINVAL for an unknown id or a range beyond n. */
pir_status pir_get_client_key(pir_server *srv, uint32_t client_id, uint32_t k0, uint32_t nk,
                              uint32_t *ck, uint32_t ptr_flags);

/* Drop a client and free its hint.  PIR_EINVAL for an unknown id. */
pir_status pir_remove_client(pir_server *srv, uint32_t client_id);

/*
 * Hint (Alg. 5): bring H up to date for every stale row, then compute
 * K_j = prod_k ck_k^{(-H_jk) mod 2^32} mod N^2 for the listed rows of this client
 * (rows == NULL or nrows == 0: all rows).  The result stays in device memory.  The
 * exponentiation uses a fixed-base table of ck powers (Alg. 4 taken to 8- or 11-bit windows,
 * see pir_hint_window_bits), built for the call and freed after it.  Row indices must be < rows (PIR_EINVAL otherwise).
 * Synchronizes the stream.
 */
pir_status pir_hint(pir_server *srv, uint32_t client_id, const uint32_t *rows, uint32_t nrows);

/*
 * Replace rows of D (the paper's silent database update, Sec. 6).  new_rows is nrows x cols
 * uint8.  Marks those rows of H and of every client's K stale; pir_compress then returns
 * PIR_ESTALE for a client until pir_hint has refreshed them.  Rows must be distinct and < rows.
 */
pir_status pir_update_rows(pir_server *srv, const uint32_t *rows, uint32_t nrows,
                           const uint8_t *new_rows, uint32_t ptr_flags);

/*
 * Memory layout of D for the batched contraction (the Alg. 5 response over many queries, and
 * H = D.A of the hint).  The server keeps D row-major (rows x pitch, pitch = cols rounded up to
 * 256) and, by default, a second copy in 16-row x 64-byte tiles: byte (j, i) at
 * (j/16) 16 pitch + (i/64) 1024 + (j mod 16) 64 + i mod 64, so that each group of 16 rows is
 * one contiguous run over its whole width.  The contraction reads the tiled copy when there
 * is one, and D otherwise; both give identical bits.  The copy costs as much HBM as D.
 * pir_setup makes it when at least an eighth of the device's memory (and 4 GiB) stays free
 * after it; pir_update_rows keeps it current.
 *   pir_set_tiled_copy: enable != 0 makes it (PIR_ENOMEM if it does not fit), 0 frees it.
 *     Synchronizes the server's stream.
 *   pir_tiled_copy: 1 if the server has it, else 0 (also for NULL).
 */
pir_status pir_set_tiled_copy(pir_server *srv, int32_t enable);
int32_t pir_tiled_copy(const pir_server *srv);

/*
 * Response, first line (Alg. 5): B[c] = D.Q[c] mod 2^32 for c < batch.
 *   Q  batch x cols uint32 (each query contiguous).   B  batch x rows uint32 (each answer contiguous).
 * batch in [1, 1024].  PIR_PATH_AUTO picks the matvec for one query and the int8-MFMA
 * byte-plane contraction otherwise; both give identical bits.
 */
pir_status pir_answer(pir_server *srv, const uint32_t *Q, uint32_t batch, uint32_t *B,
                      uint32_t ptr_flags);
pir_status pir_answer_path(pir_server *srv, const uint32_t *Q, uint32_t batch, uint32_t *B,
                           uint32_t ptr_flags, int32_t path);

/*
 * Combined response (Sec. 4.3): C[c][j] = K_{c}[j] * (1 + B[c][j] * N_c) mod N_c^2, canonical in
 * [0, N_c^2), for c < batch and j < rows.  client_ids is a host array of batch ids; every
 * client in one call must use the same limb count L.  B is batch x rows uint32 (as written by
 * pir_answer); C is batch x rows x L uint32.  PIR_ESTALE if any row of a client's hint is
 * missing or stale.
 */
pir_status pir_compress(pir_server *srv, const uint32_t *client_ids, uint32_t batch,
                        const uint32_t *B, uint32_t *C, uint32_t ptr_flags);

/*
 * One query of one client, answered and combined in one call (Alg. 5 Response, first line,
 * then the Sec. 4.3 Paillier addition): B = D.Q mod 2^32 and C[j] = K[j] (1 + B[j] N) mod N^2,
 * the same bits as pir_answer followed by pir_compress.  Q is cols uint32, B rows uint32, C
 * rows x L uint32.  The device runs two launches instead of three (the query's byte planes are
 * built inside the matvec, and the per-segment partial sums are added up by the combine).
 * PIR_EINVAL for an unknown client or a database wider than 262144 columns (use pir_answer and
 * pir_compress there); PIR_ESTALE as pir_compress.
 */
pir_status pir_answer_compress(pir_server *srv, const uint32_t *Q, uint32_t client_id, uint32_t *B,
                               uint32_t *C, uint32_t ptr_flags);

/*
 * pir_answer_compress for callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same two
 * launches and the same bits, with no hipMalloc, hipFree or allocating library call.  The
 * matvec's per-(row, column segment) partial sums go to a static array of the library on each
 * GPU (16 MiB, held until the process ends) instead of server-owned scratch.
 *   Q  cols uint32, device memory, 16-byte aligned.   B  rows uint32.   C  rows x L uint32.
 *   All three are device pointers on the server's device; there is no ptr_flags argument.
 * Limit: rows x ceil(pitch / 4096) <= 4194304 partial words (pitch = cols rounded up to 256),
 * e.g. 131072 rows at up to 131072 columns.  Beyond it, or for a misaligned Q: PIR_EINVAL.
 * Otherwise the errors of pir_answer_compress.  Returns once the work is enqueued.
 * Every call on one GPU shares that GPU's array and fully overwrites the part it uses, so
 * calls whose work overlaps on the device (different streams or servers on the same GPU, or
 * threads) race on it: serialize them.
 */
pir_status pir_answer_compress_noalloc(pir_server *srv, const uint32_t *Q, uint32_t client_id,
                                       uint32_t *B, uint32_t *C);

/*
 * Packed responses: batched compression (Alg. 3, Sec. 3.3; in ZipPIR, Sec. 4.3 "Batched
 * compression for smaller responses").  With packing factor ell, rows g*ell .. g*ell+ell-1
 * share one ciphertext
 *     C_g = prod_j c_{g ell + j}^(gamma^j) mod N^2,   c_r = K_r (1 + B[r] N) mod N^2,
 * whose plaintext holds the rows' plaintexts as base-gamma digits.  gamma = 2^t with
 * t = 64 + bitlen(n), the smallest power of two >= q + n q^2 (q = 2^32); Theorem 2 of the paper
 * holds for any gamma >= q + n q^2 and needs N > gamma^ell, so ell <= (N_bits - 1) / t.
 *
 * pir_set_packing: ell in [1, ell_max] (1 = one ciphertext per row, the default).  The group
 *   keys are derived from the client's hint: immediately if it is complete, else by the next
 *   pir_hint.  pir_update_rows marks the affected groups stale.
 * pir_packing_info: current ell, its maximum, t = log2(gamma), and the group count
 *   ceil(rows / ell) (any pointer may be NULL).
 * pir_compress_packed: C is batch x groups x L uint32 (the last group may hold fewer rows);
 *   every client in the call must have the same ell > 1 and L.  PIR_ESTALE if a row or group
 *   is stale.
 */
pir_status pir_set_packing(pir_server *srv, uint32_t client_id, uint32_t ell);
pir_status pir_packing_info(pir_server *srv, uint32_t client_id, uint32_t *ell, uint32_t *ell_max,
                            uint32_t *log2_gamma, uint32_t *groups);
pir_status pir_compress_packed(pir_server *srv, const uint32_t *client_ids, uint32_t batch,
                               const uint32_t *B, uint32_t *C, uint32_t ptr_flags);

/*
 * The paper's full protocol (Alg. 5; Sec. 4.3 "Faster matrix multiplication using RNS",
 * "Lowering offline communication costs").  The client registers random ciphertexts ck_r
 * as its key (pir_add_client), so pir_hint computes k_j = prod_k ck_r,k^{E_jk} mod N^2, and
 * sends online the offset ck_o = (s - Dec(ck_r)) mod N beside the LWE query.
 *
 * pir_offset_answer (Alg. 5 Response, second line):
 *     T[c][j] = (B[c][j] + sum_k E_jk CKO[c][k]) mod N_c,   E = (-H) mod 2^32,
 *   CKO is batch x n x h uint32 (entry k of client c's offset as h little-endian limbs; any
 *   value below 2^(32 h)), B is batch x rows uint32 (pir_answer's output), T is
 *   batch x rows x h uint32, canonical in [0, N_c).  Computes the global hint first if it is
 *   missing or stale (as pir_hint does).  Needs n <= 16384; every client in one call must use
 *   the same limb count h; batch <= 128.  Uses device scratch of about
 *   rows x batch x (16 h + 16) bytes.
 *   The client finishes with mu = (T + Dec(k_j)) mod N (Alg. 5 Extract).
 * pir_compress_offset (Sec. 4.3 "Smaller responses w/ Paillier addition" applied to t):
 *     C[c][j] = k_{c,j} (1 + T[c][j] N_c) mod N_c^2,
 *   T as written by pir_offset_answer, C batch x rows x L uint32; then mu = Dec(C).
 *   PIR_ESTALE if a client's hint has stale rows.
 */
pir_status pir_offset_answer(pir_server *srv, const uint32_t *client_ids, uint32_t batch,
                             const uint32_t *CKO, const uint32_t *B, uint32_t *T,
                             uint32_t ptr_flags);

/*
 * The full protocol's online step for one query per client in one call (Alg. 5, Response, both
 * lines): B[c] = D.Q[c] mod 2^32 (as pir_answer) and T[c] = (B[c] + E.CKO[c]) mod N_c (as
 * pir_offset_answer), the same bits as those two calls.  The offset contraction E.CKO does not
 * depend on B, so it runs on a second stream of the server (default priority) while the answer
 * runs on the server's stream; the fold of B into T waits for both.
 *   client_ids  host array of batch ids (batch in [1, 128], one shared limb count h).
 *   Q   batch x cols uint32.  CKO  batch x n x h uint32.  B  batch x rows uint32 (output).
 *   T   batch x rows x h uint32 (output, canonical residues mod N_c).
 * Errors as pir_offset_answer and pir_answer.  Device outputs: returns once enqueued on the
 * server's stream (which then orders after the second stream's work).
 */
pir_status pir_answer_offset(pir_server *srv, const uint32_t *client_ids, uint32_t batch, const uint32_t *Q,
                             const uint32_t *CKO, uint32_t *B, uint32_t *T, uint32_t ptr_flags);
pir_status pir_compress_offset(pir_server *srv, const uint32_t *client_ids, uint32_t batch,
                               const uint32_t *T, uint32_t *C, uint32_t ptr_flags);

/*
 * The full protocol with batched compression (Sec. 4.3 "Batched compression for smaller
 * responses", Theorem 2): for clients with packing factor ell > 1 (pir_set_packing), the
 * rows of a group share the key k_g = prod_j k_{g ell + j}^(gamma^j) (the packed group key) and
 * one offset answer
 *     Tg[c][g] = sum_j gamma^j t_{g ell + j} mod N_c,   gamma = 2^t (pir_packing_info),
 * where t_j is pir_offset_answer's row value.  The client computes (Tg + Dec(k_g)) mod N and
 * splits it into base-gamma digits, one per row.
 * pir_offset_answer_packed: CKO and B as for pir_offset_answer; Tg is batch x groups x h.
 *   Every client in one call must have the same ell > 1 and h.
 * pir_compress_offset_packed: Cg[c][g] = k_g (1 + Tg[c][g] N) mod N^2 (batch x groups x L);
 *   PIR_ESTALE if a hint row or group is stale.
 */
pir_status pir_offset_answer_packed(pir_server *srv, const uint32_t *client_ids, uint32_t batch,
                                    const uint32_t *CKO, const uint32_t *B, uint32_t *Tg,
                                    uint32_t ptr_flags);
pir_status pir_compress_offset_packed(pir_server *srv, const uint32_t *client_ids, uint32_t batch,
                                      const uint32_t *Tg, uint32_t *Cg, uint32_t ptr_flags);

/*
 * Standalone compression of LWE ciphertexts (Sec. 3.1, Alg. 2) and of RLWE coefficients
 * (appendix B, Alg. 8) into Paillier ciphertexts, with a resident compression key.
 *
 * A pir_compressor holds the key ck (n entries, ck[i] = Enc(s_i)) of one Paillier modulus N
 * and an LWE modulus q (2 <= q <= 2^64; pass q = 0 for 2^64).  Creation checks Theorem 1's
 * bound N > q + n (q-1)^2 and builds a fixed-base table of n x ceil(bits(q-1)/8) x 255
 * Montgomery residues on the device (about 1 GB for n = 630, q = 2^64, 3072-bit N).
 *
 * pir_compressor_create: ck is n x L uint32 (L = 2 ceil(N_bits/32), little-endian, each below
 *   N^2).  stream: a hipStream_t (NULL: the default stream).
 * pir_compressor_create_packed: the key is given packed (Sec. 3.2, Alg. 6): pck holds
 *   ceil(n/t) ciphertexts of t secret digits each, scaled for unpacking with
 *   delta = 2^delta_log2, and the device unpacks ck[it+j] = pck_i^(delta^(t-1-j)).  The client
 *   then decrypts with Alg. 6's ModifiedLWEDecryptPackedKey.
 * pir_compress_lwe: X[r] = (1 + B[r] N) prod_i ck_i^((q - A[r][i]) mod q) mod N^2 for
 *   r < rows.  A is rows x n entries and B rows entries; an entry is one uint32 when
 *   q <= 2^32, else two (little-endian uint64); entries are reduced mod q.  X is rows x L.
 * pir_compress_rlwe: for an RLWE ciphertext (A, B) over Z_q[X]/(X^n + 1) (A and B: n
 *   entries each), X[j] is the compressed coefficient ks[j] (ks: host array of nk indices
 *   below n), exponents (q - A[k-i]) mod q for i <= k and A[n+k-i] mod q for i > k.
 * pir_compressor_key: copies key entries [k0, k0+nk) (e.g. the unpacked key) into ck.
 * pir_compressor_info: L, exponent windows, device bytes held (any pointer may be NULL).
 * One ciphertext is spread over up to 256 wavefronts when few are compressed, so a single
 * compression is a short tree of Montgomery products rather than n x 8 sequential ones.
 */
typedef struct pir_compressor pir_compressor;
pir_status pir_compressor_create(pir_compressor **out, int device, void *hip_stream, uint32_t n,
                                 uint64_t q, const uint32_t *N, uint32_t N_bits,
                                 const uint32_t *ck, uint32_t ptr_flags);
pir_status pir_compressor_create_packed(pir_compressor **out, int device, void *hip_stream,
                                        uint32_t n, uint64_t q, const uint32_t *N,
                                        uint32_t N_bits, const uint32_t *pck, uint32_t t,
                                        uint32_t delta_log2, uint32_t ptr_flags);
void pir_compressor_destroy(pir_compressor *cmp);
pir_status pir_compressor_key(pir_compressor *cmp, uint32_t k0, uint32_t nk, uint32_t *ck,
                              uint32_t ptr_flags);
pir_status pir_compressor_info(pir_compressor *cmp, uint32_t *L, uint32_t *windows,
                               uint64_t *device_bytes);
/* Device time of the compressor's setup, from events on its stream: the unpacking of a packed
 * key (Alg. 6; 0 for an unpacked key) and the fixed-base table build, in milliseconds (either
 * pointer may be NULL).  Table 3 reports the unpacking time. */
pir_status pir_compressor_setup_ms(const pir_compressor *cmp, float *unpack_ms, float *table_ms);
pir_status pir_compress_lwe(pir_compressor *cmp, const uint32_t *A, const uint32_t *B,
                            uint32_t rows, uint32_t *X, uint32_t ptr_flags);
pir_status pir_compress_rlwe(pir_compressor *cmp, const uint32_t *A, const uint32_t *B,
                             const uint32_t *ks, uint32_t nk, uint32_t *X, uint32_t ptr_flags);

/* Copy rows [row0, row0+nrows) of H (nrows x n uint32).  PIR_ESTALE if any is stale. */
pir_status pir_get_global_hint(pir_server *srv, uint32_t row0, uint32_t nrows, uint32_t *H,
                               uint32_t ptr_flags);

/* Copy rows [row0, row0+nrows) of a client's hint K (nrows x L uint32) -- what a client
 * downloads in the client-storage variant (Sec. 4.3).  PIR_ESTALE if any is stale. */
pir_status pir_get_client_hint(pir_server *srv, uint32_t client_id, uint32_t row0,
                               uint32_t nrows, uint32_t *K, uint32_t ptr_flags);

/* Limb count L of a client's ciphertexts (0 for an unknown id). */
uint32_t pir_client_limbs(pir_server *srv, uint32_t client_id);

/* Window width in bits of the fixed-base table used by the client's last pir_hint (the
   exponentiation method of the Alg. 4 precomputation taken to wider windows: 8 or 11),
   0 before the first pir_hint or for an unknown id.  The result does not depend on it. */
uint32_t pir_hint_window_bits(pir_server *srv, uint32_t client_id);

/* Number of stale rows in H (client_id == UINT32_MAX) or in a client's hint. */
int64_t pir_stale_rows(pir_server *srv, uint32_t client_id);

/* Shapes of a server: rows, cols, n, and device bytes it currently owns. */
pir_status pir_shape(pir_server *srv, uint32_t *rows, uint32_t *cols, uint32_t *n,
                     uint64_t *device_bytes);

/*
 * Per-kernel timing with HIP events recorded on the server's stream around each launch of
 * the named kernels.  pir_profile(srv, 1) starts (and clears) the record, pir_profile(srv, 0)
 * stops it.  pir_profile_read synchronizes the stream and returns the summed duration in
 * milliseconds and the launch count of one kernel since profiling started.
 */
#define PIR_KERNEL_MATVEC   0  /* one-query answer (u8 x u32 dot4 stream)               */
#define PIR_KERNEL_GEMM     1  /* byte-plane int8-MFMA contraction (batched answer, H)  */
#define PIR_KERNEL_COMPRESS 2  /* per-row Paillier combine                              */
#define PIR_KERNEL_HINT     3  /* per-row fixed-base multi-exponentiation               */
#define PIR_KERNEL_TABLE    4  /* fixed-base table build                                */
#define PIR_KERNEL_KEY      5  /* per-row combine key N (K mod N), computed with the hint */
#define PIR_KERNEL_OFFSET_GEMM 6  /* offset answer: E bytes x offset bytes on int8 MFMA   */
#define PIR_KERNEL_OFFSET   7  /* offset answer: byte positions -> limbs, + b, mod N     */
#define PIR_KERNEL_STEP_MATVEC  8  /* pir_answer_compress: matvec into segment partials   */
#define PIR_KERNEL_STEP_COMBINE 9  /* pir_answer_compress: partials -> b, Paillier combine */
#define PIR_KERNEL_COUNT    10
pir_status pir_profile(pir_server *srv, int32_t enable);
pir_status pir_profile_read(pir_server *srv, int32_t kernel, double *total_ms, uint64_t *launches);

/* Wait for all work the server enqueued. */
pir_status pir_sync(pir_server *srv);

/* Static description of a status code. */
const char *pir_strerror(pir_status st);

/* Detail of the last failure on the calling thread ("" if none). */
const char *pir_last_error(void);

/* ============================================================================
 * Serving engine: continuous batching over several resident databases.
 *
 * Clients issue many queries, each answered with its own resident hint (Sec. 4.3,
 * "Supporting multiple queries"); D, A and H are shared by all clients.  The engine owns a
 * scheduler thread.  Requests for one database wait in a FIFO queue; whenever that
 * database has a free slot (at most two batches in flight per database) the scheduler
 * takes up to max_batch queued requests whose clients share a limb count, runs
 * pir_answer (batch 1: matvec; larger: one int8-MFMA contraction) and pir_compress on the
 * database's stream, and copies each compressed response into the caller's buffer.
 * Batches of different databases run on different streams and overlap on the device.  A
 * batch is enqueued in steps (the answer in row ranges of at most step_bytes of D, each
 * response's download in pieces of at most copy_bytes); with more than one database
 * registered, at most two steps of a batch are queued on the device at a time, so a small
 * database's request waits for at most a couple of a large database's steps.
 * Device buffers for in-flight batches are admitted against a byte budget: a batch that
 * does not fit waits until earlier batches complete.  Buffers are reused through a pool and
 * freed only when the budget cannot otherwise admit a batch.  Results do not depend on how
 * requests were batched or stepped.
 * ==========================================================================*/
typedef struct pir_engine pir_engine;

typedef struct pir_completion {
  uint64_t request_id;
  uint32_t db;          /* engine database index                                   */
  uint32_t client_id;
  int32_t status;       /* PIR_OK or the status of the batch the request ran in    */
  uint32_t batch;       /* number of requests in that batch                        */
  double arrival_ms;    /* engine clock (ms since pir_engine_create): arrival       */
  double start_ms;      /* batch enqueued on the device                             */
  double done_ms;       /* response written to the caller's buffer                  */
} pir_completion;

typedef struct pir_engine_stats {
  uint64_t submitted, completed, failed, batches;
  uint64_t admission_waits;   /* times a formed batch waited for device budget          */
  uint64_t device_bytes_peak; /* peak bytes of in-flight batch buffers                  */
  double p50_ms, p99_ms;      /* latency = done - arrival over completed requests       */
  double mean_batch;
} pir_engine_stats;

/* max_batch in [1, 1024].  hbm_budget_bytes: device bytes the engine may hold for in-flight
 * batches (0: the device's free memory at creation minus 1 GiB). */
pir_status pir_engine_create(pir_engine **out, uint32_t max_batch, uint64_t hbm_budget_bytes);

/* Step sizes of a batch: bytes of D per answer step (rounded down to a multiple of 256 rows,
 * at least 256 rows; default 256 MiB) and response bytes per download step (default 8 MiB).
 * Only before the first pir_engine_add_db (PIR_EINVAL after it, or for 0). */
pir_status pir_engine_set_steps(pir_engine *eng, uint64_t step_bytes, uint64_t copy_bytes);

/* Register a database.  The server must have been set up with its own stream (not NULL); from
 * now until pir_engine_destroy only the engine may use it.  The call runs the batched answer
 * once for each column-group shape up to max_batch (on zero queries, in the engine's row
 * steps) so that those contraction shapes are tuned and their scratch sized now; while the
 * server is registered, a shape not tuned yet runs with the default launch shape instead of
 * being tuned in place. */
pir_status pir_engine_add_db(pir_engine *eng, pir_server *srv, uint32_t *db_index);

/* Queue one request.  query: host array of the database's cols uint32 (copied before the call
 * returns).  result: rows x L uint32 in pinned host memory (pir_host_alloc) or device memory,
 * or groups x L (groups = ceil(rows / ell)) when the client has packed responses
 * (pir_set_packing; the packing factor is read here, so it must not change while the
 * client's requests are queued); it must stay valid until the request's completion is
 * returned by pir_engine_poll.
 * arrival_ms: engine-clock time before which the request is not started (< 0: now).
 * Errors: PIR_EINVAL (unknown database or client, pageable result buffer). */
pir_status pir_engine_submit(pir_engine *eng, uint32_t db_index, uint32_t client_id,
                             const uint32_t *query, uint32_t *result, double arrival_ms,
                             uint64_t *request_id);

/* Up to max completions, oldest first; waits up to timeout_ms (0: do not wait) for one. */
pir_status pir_engine_poll(pir_engine *eng, pir_completion *out, uint32_t max, uint32_t *count,
                           int32_t timeout_ms);

/* Wait until every submitted request has completed (PIR_EBUSY on timeout; < 0: no limit). */
pir_status pir_engine_drain(pir_engine *eng, int32_t timeout_ms);

pir_status pir_engine_stats_get(pir_engine *eng, pir_engine_stats *st);

/* Engine clock now (ms since creation). */
double pir_engine_now_ms(pir_engine *eng);

/* Stops the scheduler after in-flight work completes and frees the engine's buffers (the
 * servers stay alive and usable again). */
void pir_engine_destroy(pir_engine *eng);

/* Admission policy, exposed for testing.  pir_engine_capacity: how many requests' buffers
 * (bytes_per_request each) fit in budget_free, at most max_batch.  pir_engine_plan: how many
 * leading queued requests form the next batch: those sharing the first one's batch key (the
 * engine uses limb count | packing factor << 16), at most capacity. */
uint32_t pir_engine_capacity(uint64_t budget_free, uint64_t bytes_per_request, uint32_t max_batch);
uint32_t pir_engine_plan(const uint32_t *queued_limbs, uint32_t nqueued, uint32_t capacity);

/*
 * Streaming-read probe (measurement only): reads the first bytes - bytes mod 16 bytes of the
 * device buffer buf (16-byte aligned) once with nontemporal loads, `blocks` workgroups of 256
 * threads, each streaming its own contiguous chunk of about bytes / blocks bytes, and writes
 * one word per workgroup to sink (a device array of `blocks` words).
 * Enqueued on hip_stream; the time of this launch gives the device's achievable HBM read
 * bandwidth, the practical ceiling of the one-query answer.
 */
pir_status pir_read_probe(const void *buf, uint64_t bytes, uint32_t *sink, uint32_t blocks,
                          void *hip_stream);

/* Pinned host memory for engine results (NULL on failure). */
void *pir_host_alloc(uint64_t bytes);
void pir_host_free(void *p);

#ifdef __cplusplus
}
#endif

#endif /* ZIPPIR_H */
