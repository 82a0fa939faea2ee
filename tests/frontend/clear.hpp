// Cleartext build of the front end's test programs: word_t is an element of F_p, p = 2^32 - 5,
// with the ring operations of the field and the integer order of its canonical representative
// (public comparisons); mark_linear_layer computes W x + b.  Test infrastructure only.
#include <stdint.h>
struct Fp {
  uint64_t v;
  static constexpr uint64_t P = 4294967291ull;
  Fp() : v(0) {}
  Fp(long long c) : v(c >= 0 ? (uint64_t)c % P : (P - (uint64_t)(-c) % P) % P) {}
  Fp(unsigned long long c) : v(c % P) {}
  Fp(int c) : Fp((long long)c) {}
  Fp(unsigned c) : Fp((unsigned long long)c) {}
  Fp(long c) : Fp((long long)c) {}
  Fp(unsigned long c) : Fp((unsigned long long)c) {}
};
inline Fp operator+(Fp a, Fp b) { Fp r; r.v = (a.v + b.v) % Fp::P; return r; }
inline Fp operator-(Fp a, Fp b) { Fp r; r.v = (a.v + Fp::P - b.v) % Fp::P; return r; }
inline Fp operator*(Fp a, Fp b) { Fp r; r.v = (uint64_t)((unsigned __int128)a.v * b.v % Fp::P); return r; }
inline Fp operator<<(Fp a, int k) { return a * Fp((unsigned long long)1 << k); }
inline Fp &operator+=(Fp &a, Fp b) { return a = a + b; }
inline Fp &operator-=(Fp &a, Fp b) { return a = a - b; }
inline Fp &operator*=(Fp &a, Fp b) { return a = a * b; }
inline bool operator<(Fp a, Fp b) { return a.v < b.v; }
inline bool operator>(Fp a, Fp b) { return a.v > b.v; }
typedef Fp word_t;
#define SPDZ_PRIVATE
#define SPDZ_PUBLIC
static word_t layer_out[1 << 16];
inline word_t *mark_linear_layer(const word_t *x, const word_t *W, const word_t *b, int din, int dout) {
  for (int r = 0; r < dout; r++) {
    word_t s = b[r];
    for (int k = 0; k < din; k++) s += W[(long)r * din + k] * x[k];
    layer_out[r] = s;
  }
  return layer_out;
}
