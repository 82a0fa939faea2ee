/* Programs the front end must refuse. */
word_t secret_branch(const word_t *x SPDZ_PRIVATE) {
    word_t r = 0;
    for (int i = 0; i < 8; i++) {
        if (x[i] < 100) r += x[i];
        else r += x[i] * x[i];
    }
    return r;
}
void stores(const word_t *x SPDZ_PRIVATE, word_t *out) {
    for (int i = 0; i < 16; i++) out[i] = x[i] * x[i];
}
word_t secret_shift(const word_t *x SPDZ_PRIVATE) {
    return (x[0] >> 3) + x[1];
}
word_t secret_mask(const word_t *x SPDZ_PRIVATE) {
    return (x[0] & 255u) * x[1];
}
word_t public_odd_mask(const word_t *x SPDZ_PRIVATE, uint32_t n SPDZ_PUBLIC) {
    word_t acc = 0;
    for (uint32_t i = 0; i < (n & 0x55u); i++) acc += x[i];
    return acc;
}
