"""Seeded random C functions for the front end's tests (test infrastructure only).

    word_t fz(const word_t *x SPDZ_PRIVATE, const word_t *y SPDZ_PRIVATE,
              word_t s SPDZ_PRIVATE, uint32_t t SPDZ_PUBLIC)

x and y point to `n` elements.  The body mixes straight-line +, -, * on private values and odd
literals, dot-product loops the vectorizer turns into vector reductions, Horner-style loops it
cannot vectorize, if/else and ?: on public comparisons of t, and loops whose trip count is a
low-bit mask of t.  No shifts, only odd constants and no value added to itself or appearing twice in the returned
sum: the C function and its translation agree in F_p only while clang's bit-level reasoning
about 32-bit integers has nothing to act on (known trailing zeros of a product; or, where a value
is only ever used doubled, constants feeding it rewritten modulo 2^31).
"""
import random


def random_c(seed: int, n: int = 64, statements: int = 8) -> str:
    rng = random.Random(seed)
    body, names = [], []

    def leaf(allow_const=True):
        r = rng.random()
        if r < 0.35 and names:
            return rng.choice(names)
        if r < 0.6:
            return f"x[{rng.randrange(n)}]"
        if r < 0.82:
            return f"y[{rng.randrange(n)}]"
        if r < 0.9 or not allow_const:
            return "s"
        return str(rng.choice([1, 3, 5, 7, 9, 11, 13, 101, 1001]))

    def binexpr():
        a, b = leaf(), leaf(allow_const=False)
        op = rng.choice(['+', '-', '*'])
        if a == b and op == "+":   # a + a doubles a
            op = "*"
        return f"{a} {op} {b}"

    def new_name():
        v = f"v{len(names)}"
        names.append(v)
        return v

    for _ in range(statements):
        r = rng.random()
        if r < 0.25 or not names:
            e = binexpr()
            body.append(f"word_t {new_name()} = {e};")
        elif r < 0.40:
            v, w = rng.choice(names), leaf()
            op = rng.choice(['+', '-', '*'])
            if w == v and op == "+":
                op = "*"
            body.append(f"{v} = {v} {op} {w};")
        elif r < 0.55:
            init = leaf()
            v = new_name()
            L = rng.choice([8, 16, 24, n])
            op = rng.choice(["*", "+", "-"])
            c = rng.choice(["", f" * {rng.choice([3, 5, 7])}"])
            body.append(f"word_t {v} = {init};")
            body.append(f"for (int i = 0; i < {L}; i++) {v} += x[i] {op} y[i]{c};")
        elif r < 0.65:
            init = leaf()
            v = new_name()
            L = rng.randint(2, 10)
            body.append(f"word_t {v} = {init};")
            body.append(f"for (int i = 0; i < {L}; i++) {v} = {v} * x[i] + y[i];")
        elif r < 0.78:
            v = rng.choice(names)
            body.append(f"if (t < {rng.randrange(1, 200)}u) {{ {v} = {binexpr()}; }} else {{ {v} = {binexpr()}; }}")
        elif r < 0.88:
            v = rng.choice(names)
            body.append(f"{v} = t > {rng.randrange(1, 200)}u ? {leaf()} : {leaf()};")
        else:
            init = leaf()
            v = new_name()
            mask = rng.choice([7, 15, 31])
            body.append(f"word_t {v} = {init};")
            body.append(f"for (uint32_t i = 0; i < (t & {mask}u); i++) {v} += x[i] * y[i];")
    if len(names) >= 3:
        ret = f"{names[-1]} * {names[-2]} + {names[-3]}"
    elif len(names) == 2:
        ret = f"{names[-1]} * {names[-2]}"
    else:
        ret = names[-1]
    src = ["word_t fz(const word_t *x SPDZ_PRIVATE, const word_t *y SPDZ_PRIVATE, word_t s SPDZ_PRIVATE,",
           "          uint32_t t SPDZ_PUBLIC) {"]
    src += ["    " + b for b in body]
    src += [f"    return {ret} + s;", "}"]
    return "\n".join(src) + "\n"
