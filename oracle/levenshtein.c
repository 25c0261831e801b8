/* Textbook Levenshtein distance (unit-cost insertion, deletion, substitution),
 * the edit distance named in the RotorMap paper's introduction (§1).
 *
 * TEST INFRASTRUCTURE ONLY: part of the FP64/CPU oracle.  Built by the
 * package build step into oracle/_liblev.so and called through ctypes by
 * oracle/lev.py.
 *
 * D[i][j] = min(D[i-1][j] + 1, D[i][j-1] + 1, D[i-1][j-1] + [a_i != b_j]),
 * D[i][0] = i, D[0][j] = j; computed one row at a time.
 */
#include <stdint.h>
#include <stdlib.h>

static int64_t lev_one(const uint8_t* a, int64_t na, const uint8_t* b, int64_t nb, int64_t* row) {
  for (int64_t j = 0; j <= nb; ++j) row[j] = j;
  for (int64_t i = 1; i <= na; ++i) {
    int64_t diag = row[0];
    row[0] = i;
    for (int64_t j = 1; j <= nb; ++j) {
      int64_t up = row[j];
      int64_t best = up + 1;
      if (row[j - 1] + 1 < best) best = row[j - 1] + 1;
      int64_t sub = diag + (a[i - 1] != b[j - 1]);
      if (sub < best) best = sub;
      diag = up;
      row[j] = best;
    }
  }
  return row[nb];
}

/* Distances of n pairs; pair i is a[a_off[i]:a_off[i+1]] vs b[b_off[i]:b_off[i+1]].
 * Returns 0, or -1 if scratch memory could not be allocated. */
int lev_many(const uint8_t* a, const int64_t* a_off, const uint8_t* b, const int64_t* b_off,
             int64_t n, int64_t* out) {
  int64_t maxb = 0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t nb = b_off[i + 1] - b_off[i];
    if (nb > maxb) maxb = nb;
  }
  int64_t* row = (int64_t*)malloc(sizeof(int64_t) * (size_t)(maxb + 1));
  if (!row) return -1;
  for (int64_t i = 0; i < n; ++i)
    out[i] = lev_one(a + a_off[i], a_off[i + 1] - a_off[i], b + b_off[i], b_off[i + 1] - b_off[i], row);
  free(row);
  return 0;
}
