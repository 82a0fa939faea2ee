/*
 * spdz_frontend.h -- declarations for C programs compiled by the LLVM front end
 * (paper_2512_11112_amd/frontend.py), which passes this file to clang with -include.
 *
 * Parameters of the entry function carry a privacy annotation, the paper's
 * __attribute__((annotate("private"))) / __attribute__((annotate("public")))
 * (Sec. III-A, Fig. 2); SPDZ_PRIVATE and SPDZ_PUBLIC spell them.  The function
 * returns the value the parties reveal.
 *
 * mark_linear_layer is the reserved marker of an ML linear layer f = W x + b
 * (Sec. III-A, Fig. 2): x [din], W [dout][din] row-major, b [dout]; the front
 * end turns the call into one layer node of the runtime.  It has no
 * definition here: a program that calls it is only ever compiled to IR.
 */
#ifndef SPDZ_FRONTEND_H
#define SPDZ_FRONTEND_H

#include <stdint.h>

#define SPDZ_PRIVATE __attribute__((annotate("private")))
#define SPDZ_PUBLIC __attribute__((annotate("public")))

/* a 32-bit word: a residue of the field of the paper's evaluation, p = 2^32 - 5 (Sec. IV-A) */
typedef uint32_t word_t;

#ifdef __cplusplus
extern "C" {
#endif

word_t *mark_linear_layer(const word_t *x, const word_t *W, const word_t *b, int din, int dout);

#ifdef __cplusplus
}
#endif
#endif /* SPDZ_FRONTEND_H */
