/* A loop bounded by a public parameter: the sum of x[i] y[i] + 3 x[i] for i < n. */
word_t dot(const word_t *x SPDZ_PRIVATE, const word_t *y SPDZ_PRIVATE, uint32_t n SPDZ_PUBLIC) {
    word_t acc = 0;
    for (uint32_t i = 0; i < n; i++) acc += x[i] * y[i] + 3 * x[i];
    return acc;
}
