/* Straight-line arithmetic on private scalars and vector elements, a public select. */
word_t poly(const word_t *x SPDZ_PRIVATE, word_t s SPDZ_PRIVATE, uint32_t c SPDZ_PUBLIC) {
    word_t a = x[0] * x[1] + s;
    word_t b = c > 2 ? a * s : a + x[2];
    return b * b - (x[3] << 2);
}
