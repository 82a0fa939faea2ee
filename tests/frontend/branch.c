/* A branch on a public parameter, each side a loop (so the optimiser keeps the branch),
 * joined by a phi, then a product with a constant shift and an offset. */
word_t branchy(const word_t *x SPDZ_PRIVATE, const word_t *y SPDZ_PRIVATE, uint32_t t SPDZ_PUBLIC) {
    word_t acc = 0;
    if (t < 5) {
        for (int i = 0; i < 64; i++) acc += x[i] * y[i];
    } else {
        for (int i = 0; i < 64; i++) acc += x[i] - y[i];
    }
    return (acc << 3) * x[0] + 5 * y[1] - 7;
}
