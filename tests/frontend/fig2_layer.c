/* The paper's Fig. 2 program (Sec. III-A): a linear layer marked for the front end,
 * x and W private, b public.  DIN and DOUT come from the command line. */
word_t *linear_layer(const word_t *x SPDZ_PRIVATE, const word_t *W SPDZ_PRIVATE, const word_t *b SPDZ_PUBLIC) {
    word_t *out = mark_linear_layer(x, W, b, DIN, DOUT);
    return out;
}
