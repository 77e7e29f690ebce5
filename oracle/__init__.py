"""CPU oracle for the ZipPIR server path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the server computes, written from
the paper (ZipPIR: High-throughput Single-server PIR without Client-side Storage):

* ``lwe``      -- LWE encryption/decryption (Alg. 1), the PIR query and extraction (Alg. 5).
* ``paillier`` -- the Paillier cryptosystem (Sec. 2.1) with generator N+1.
* ``server``   -- the server-side parity targets: global hint H = D.A mod 2^32, exponents
                  E = (-H) mod 2^32, client hint K_j = prod_k ck_k^{E_jk} mod N^2, the
                  online answer b = D.qu mod 2^32 and the compressed row
                  c_j = K_j (+) Enc(b_j; 1) (Alg. 2, Alg. 5, Sec. 4.3).
* ``protocol`` -- the paper's full protocol (Alg. 5 with random hint keys and the online
                  offset answer t = b + E.ck_o mod N; Sec. 4.3 Paillier addition).
* ``compress`` -- standalone LWE and RLWE ciphertext compression (Alg. 2, packed keys of
                  Alg. 6, RLWE coefficients of Alg. 8).
* ``prg``      -- the seed expansion of the silent offline phase (Sec. 4.3): ChaCha20
                  (RFC 8439) and the rejection sampler of random hint keys in Z_{N^2}.
* ``brute``    -- the same quantities by pure-Python loops, for tiny sizes.
* ``params``   -- the parameter conditions (Theorem 1 of Sec. 3.1, the ZipPIR correctness
                  condition of Sec. 4.2).

Only the test-suite, the package smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never imports it.
Integer arithmetic is exact: numpy uint64 products wrap modulo 2^64, which is exact
modulo 2^32 after masking; everything modulo N^2 uses Python integers and ``pow``.
"""
from . import brute, compress, lwe, paillier, params, prg, protocol, server  # noqa: F401
