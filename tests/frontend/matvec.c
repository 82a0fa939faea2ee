/* Nested loops over a row-major matrix (no layer marker): the sum of the squared entries of
 * W x.  The optimiser unrolls and vectorizes the inner loop; the outer loop indexes the rows
 * by a byte offset (row * DIN * 4). */
word_t matvec_sum(const word_t *W SPDZ_PRIVATE, const word_t *x SPDZ_PRIVATE) {
    word_t total = 0;
    for (int r = 0; r < DOUT; r++) {
        word_t acc = 0;
        for (int k = 0; k < DIN; k++) acc += W[r * DIN + k] * x[k];
        total += acc * acc;
    }
    return total;
}
