// Beaver product kernels over 2^127 - 1.
#include "beaver.h"

namespace spdz {
template spdz_status launch_beaver_field<F127>(spdz_ctx *, const spdz_shares *, const spdz_shares *,
                                               const spdz_triple *, spdz_shares *, u64 *, u64 *, const u64 *,
                                               spdz_shares *, u64 *, spdz_shares *, u64 *);
}  // namespace spdz
