// Host-side entry points shared by the library's C++ sources (not part of the
// C ABI).
#pragma once

#include "../../include/mtgp.h"

namespace mtgp_impl {

// mtgp_batch_generate; with allow_split false a request is never turned into
// jump-ahead segments, whatever the batch's split limit (the request loop's
// ticks, whose chunks are short by construction).
int batch_generate(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream, bool allow_split);

}  // namespace mtgp_impl
