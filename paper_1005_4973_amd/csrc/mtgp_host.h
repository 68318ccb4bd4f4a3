// Host-side entry points shared by the library's C++ sources (not part of the
// C ABI).
#pragma once

#include "../../include/mtgp.h"
#include "mtgp_f2.h"
#include "mtgp_internal.h"

#include <algorithm>
#include <vector>

namespace mtgp_impl {

// Stable order of jump items by launch geometry (lane width R, then word
// groups G): the jump kernel is launched once per (R, G). Sorts (key, index)
// pairs and permutes, so no temporary JumpItem buffer (which the standard
// library need not align to 32 bytes) is made.
inline void group_jumps_by_shape(std::vector<JumpItem> &jumps)
{
    std::vector<std::pair<uint64_t, uint32_t>> key(jumps.size());
    for (size_t i = 0; i < jumps.size(); i++) {
        const JumpShape sh = jump_shape(jumps[i].N);
        key[i] = {((uint64_t)sh.R << 32) | sh.G, (uint32_t)i};
    }
    std::sort(key.begin(), key.end());
    std::vector<JumpItem> out(jumps.size());
    for (size_t i = 0; i < key.size(); i++)
        out[i] = jumps[key[i].second];
    jumps.swap(out);
}

// mtgp_batch_generate; with allow_split false a request is never turned into
// jump-ahead segments, whatever the batch's split limit (the request loop's
// ticks, whose chunks are short by construction).
int batch_generate(mtgp_batch_t *b, const mtgp_request *reqs, uint32_t nreq, void *stream, bool allow_split);

// The persistent generation over prepared work items (no request checks:
// items may share a generator when at most one of them writes its state
// back to it), on stream s; adds each item's outputs to its generator's
// consumed counter.
int launch_work_items(mtgp_batch_t *b, std::vector<WorkItem> &items, hipStream_t s);

// Jump-ahead support for the request loop. split_ready: the generator's
// orbit annihilator psi is known (prepare_annihilators computes it,
// synchronously: raw words on the device, Berlekamp-Massey on the host);
// segment_polys: h_k = x^{kJ} mod psi for k = 1 .. S-1; poly_layout writes h
// in the jump kernel's layout (poly_words(N, deg psi) words); the raw
// prefix (the N state words and deg psi - 1 new ones, state kept) runs as
// work items of kind raw under prefix_shape.
bool split_ready(const mtgp_batch_t *b, uint32_t g);
const f2::Poly &split_psi(const mtgp_batch_t *b, uint32_t g);
uint32_t gen_words(const mtgp_batch_t *b, uint32_t g);
uint32_t max_gen_words(const mtgp_batch_t *b);
int prepare_annihilators(mtgp_batch_t *b, const std::vector<uint32_t> &gens);
uint32_t poly_words(uint32_t N, uint32_t D);
void poly_layout(const f2::Poly &h, uint32_t N, uint64_t *dst);
std::vector<f2::Poly> segment_polys(const f2::Poly &psi, uint64_t J, uint32_t S);
LaunchShape prefix_shape(const mtgp_batch_t *b, const std::vector<uint32_t> &gens);
uint16_t prefix_spl(const mtgp_batch_t *b, uint32_t g, const LaunchShape &shape);
hipError_t launch_prefix(mtgp_batch_t *b, const WorkItem *d_items, uint32_t n, const LaunchShape &shape,
                         hipStream_t s);

}  // namespace mtgp_impl
