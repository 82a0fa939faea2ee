/* A secret scalar against vectors: sum_i (a x[i] + y[i])^2.  The vectorized loop repeats the
 * secret a across the lanes of a vector (a broadcast of a secret value). */
word_t axpy_dot(const word_t *x SPDZ_PRIVATE, const word_t *y SPDZ_PRIVATE, word_t a SPDZ_PRIVATE) {
    word_t acc = 0;
    for (int i = 0; i < 64; i++) {
        word_t z = a * x[i] + y[i];
        acc += z * z;
    }
    return acc;
}
