/* A loop whose bound is known only at run time: a public count taken below the arrays' length.
 * The vectorized loop's trip count is that bound rounded down to a multiple of the vector
 * length (an and with a mask); the remainder loop runs element by element. */
word_t dot_rt(const word_t *x SPDZ_PRIVATE, const word_t *y SPDZ_PRIVATE, uint32_t n SPDZ_PUBLIC) {
    uint32_t m = n % 4001u;
    word_t acc = 0;
    for (uint32_t i = 0; i < m; i++) acc += x[i] * y[i] + 3 * x[i];
    return acc;
}
