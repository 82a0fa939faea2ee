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
