/*
 * Exact CPU oracle for the modular matrix product C = A B mod p.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no source with
 * the GPU library and includes none of its headers.
 *
 * What it computes is the definition of the problem (Section 1, eq. goal):
 *     C[i][j] = ( sum_l A[i][l] * B[l][j] ) mod p
 * over the integers.  The paper's multiword method reaches exactly this value
 * (Section 3.2, Prop. UVMW), so the definition is the oracle; none of the
 * paper's floating-point steps appear here.
 *
 * Arithmetic: operands are reduced mod p first (entries may be any uint64),
 * products are formed in unsigned __int128 and summed in unsigned __int128,
 * and one "% p" is taken per output.  For p < 2^52 (the bitsizes the method
 * handles) each product is below 2^104, so sums of up to 2^24 products fit.
 * The general limit is checked: k * (p-1)^2 must fit in 128 bits, else the
 * call returns -2.
 *
 * Threads: OpenMP over output rows.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* Returns 1 if k * (p-1)^2 < 2^128. */
static int sum_fits(uint64_t p, int64_t k) {
  u128 pm = (u128)(p - 1) * (u128)(p - 1);
  if (pm == 0 || k <= 1) return 1;
  u128 limit = ~(u128)0;
  return pm <= limit / (u128)k;
}

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * C (m x n) = A (m x k) * B (k x n) mod p, all row-major uint64, host memory.
 * Returns 0 on success, -1 on bad arguments, -2 if the exact sum could
 * overflow 128 bits, -3 on allocation failure.
 */
int oracle_mm_modp(uint64_t p, int64_t m, int64_t n, int64_t k,
                   const uint64_t *A, const uint64_t *B, uint64_t *C) {
  if (p < 2 || m < 0 || n < 0 || k < 0) return -1;
  if ((m > 0 && n > 0) && (!C || (k > 0 && (!A || !B)))) return -1;
  if (!sum_fits(p, k)) return -2;
  if (m == 0 || n == 0) return 0;

  uint64_t *Ar = NULL, *Br = NULL;
  if (k > 0) {
    Ar = (uint64_t *)malloc((size_t)m * (size_t)k * sizeof(uint64_t));
    Br = (uint64_t *)malloc((size_t)k * (size_t)n * sizeof(uint64_t));
    if (!Ar || !Br) {
      free(Ar);
      free(Br);
      return -3;
    }
    for (int64_t i = 0; i < m * k; i++) Ar[i] = A[i] % p;
    for (int64_t i = 0; i < k * n; i++) Br[i] = B[i] % p;
  }

  int failed = 0;
#pragma omp parallel
  {
    u128 *acc = (u128 *)malloc((size_t)n * sizeof(u128));
    if (!acc) {
#pragma omp atomic write
      failed = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; i++) {
      if (!acc) continue;
      memset(acc, 0, (size_t)n * sizeof(u128));
      for (int64_t l = 0; l < k; l++) {
        const u128 a = (u128)Ar[i * k + l];
        const uint64_t *brow = Br + l * n;
        for (int64_t j = 0; j < n; j++) acc[j] += a * (u128)brow[j];
      }
      for (int64_t j = 0; j < n; j++) C[i * n + j] = (uint64_t)(acc[j] % (u128)p);
    }
    free(acc);
  }
  free(Ar);
  free(Br);
  return failed ? -3 : 0;
}

/*
 * Selected outputs only: C_out[t] = (row rows[t] of A) . (column cols[t] of B) mod p.
 * Used to check sampled outputs of products too large for the full oracle.
 */
int oracle_mm_modp_entries(uint64_t p, int64_t m, int64_t n, int64_t k,
                           const uint64_t *A, const uint64_t *B, int64_t count,
                           const int64_t *rows, const int64_t *cols, uint64_t *C_out) {
  if (p < 2 || m < 0 || n < 0 || k < 0 || count < 0) return -1;
  if (count > 0 && (!rows || !cols || !C_out || (k > 0 && (!A || !B)))) return -1;
  if (!sum_fits(p, k)) return -2;
  for (int64_t t = 0; t < count; t++)
    if (rows[t] < 0 || rows[t] >= m || cols[t] < 0 || cols[t] >= n) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < count; t++) {
    u128 acc = 0;
    const int64_t i = rows[t], j = cols[t];
    for (int64_t l = 0; l < k; l++)
      acc += (u128)(A[i * k + l] % p) * (u128)(B[l * n + j] % p);
    C_out[t] = (uint64_t)(acc % (u128)p);
  }
  return 0;
}
