// MTGP generation kernels for gfx950 (MI355X).
//
// One workgroup evaluates one generator at a time. Its state lives in an LDS
// window X[0..L): X[base + k] holds x_{i0 + k} for the current round start i0.
// A round computes `cnt <= W <= N - M` consecutive steps i0 .. i0+cnt-1 at
// once; they are mutually independent because step i reads x_i, x_{i+1},
// x_{i+M-1}, x_{i+M}, all older than x_{i0+N} (section 3.2: with a long
// enough array, N - M steps can run in parallel). Every read of a round is
// issued before any of its writes, the round's new words go to
// X[base + N .. base + N + cnt), and one barrier separates rounds. When the
// window reaches the end of X, the N live words are copied back to X[0..N),
// so no address ever wraps.
//
// Every lane evaluates all of its step slots in every round, without
// branches; only the output store is predicated (k < cnt). A slot beyond the
// round (k >= cnt) reads words inside the live window and writes
// X[base + N + k], a slot no step of this round reads and the next round
// overwrites before reading it. Hence the window needs L >= 2N + lanes*spl
// (source and destination of the compaction copy are then disjoint too).
// Loads of a round are issued first, then the tempering lookups, then the
// recursion's VALU work, its table lookup and the writes; the tempering
// lookups return while that work runs, so a round's chain is its loads, the
// recursion, one lookup, its writes and the barrier. Both 16-word tables
// (recursion and output) sit in LDS ahead of the window.
//
// Step k of a round is done by lane k mod T in pass k / T (T = workgroup
// size), so LDS reads and writes are unit-stride across a wavefront and the
// outputs of a pass are one contiguous, coalesced store.
//
// Per step (section 3.6 and 3.7):
//   t = x_{i+1} ^ (x_i & mask);  t ^= t << sh1;  u = t ^ (x_{i+M} >> sh2)
//   x_{i+N} = u ^ rec[u & 0xf]
//   s = x_{i+M-1} ^ (x_{i+M-1} >> 16);  s ^= s >> 8
//   uint32:      o = x_{i+N} ^ tmp[s & 0xf]
//   float [1,2): o = (x_{i+N} >> 9) ^ flt[s & 0xf]       (section 6, eq. (C))
//   float [0,1): the [1,2) value minus 1.0f
//   normal:      Box-Muller on the pair of float [1,2) outputs (a, b) at
//                positions 2j, 2j+1 of the call: r = sqrt(-2 ln(2 - a)),
//                output 2j = r cos(2 pi (b - 1)), output 2j+1 = r sin(...);
//                section 6 names [1,2) as the input for this transform
//                (evaluated with the hardware log2, sqrt and sine)
#include "mtgp_internal.h"

#include <mutex>

namespace mtgp_impl {

// LDS layout: [0,16) recursion table, [16,32) output table, [32] queue slot,
// window X from word 64 on.
constexpr uint32_t kTableWords = 64;

// Outputs are written with buffer stores (see out_window): unlike flat
// stores they count on vmcnt only, so the LDS wait before each round's
// barrier never waits for HBM write acknowledgements.
typedef uint32_t gu32;

template <int KIND>
__device__ __forceinline__ uint32_t output_word(uint32_t x, uint32_t tv)
{
    if constexpr (KIND == kKindU32) {
        return x ^ tv;
    } else if constexpr (KIND == kKindRaw) {
        return x;   // untempered word (input of the jump correlation)
    } else {
        const uint32_t b = (x >> 9) ^ tv;
        if constexpr (KIND == kKindF01) {
            return __float_as_uint(__uint_as_float(b) - 1.0f);
        } else {
            return b;   // float [1,2); the normal kind transforms it in pairs
        }
    }
}

// DPP controls quad_perm(0,0,2,2) and quad_perm(1,1,3,3): lanes 2m and 2m+1
// both read lane 2m, or both read lane 2m+1.
constexpr int kDppPairFirst = 0xa0;
constexpr int kDppPairSecond = 0xf5;

// -2 ln 2: r^2 = -2 ln(u1) = -2 ln 2 * log2(u1)
constexpr float kMinus2Ln2 = -1.3862943611198906f;

// Box-Muller on the float [1,2) bits `f` of this lane and of its pair
// partner (lane ^ 1); the even lane holds the first of the pair, a, and
// returns r cos(theta), the odd lane r sin(theta). Both lanes of a pair read
// a and b from the pair's lanes (a DPP broadcast within the pair). 2 - a is
// exact in binary32, so the logarithm's argument lies in (0, 1]; the angle is
// taken in revolutions by the hardware sine (input t means sin(2 pi t)), with
// t = b - 1 for the sine and t = b - 3/4 = (b - 1) + 1/4 for the cosine
// (cos(2 pi x) = sin(2 pi (x + 1/4))); both are exact, multiples of 2^-23
// in [0, 1.25). The hardware base-2 logarithm, square root and sine are used
// directly: over all 2^23 inputs of each, r is within 4.7e-7 and the sine and
// cosine within 1.3e-7 of the exact values (measured exhaustively on gfx950),
// so |z| is within about 1.5e-6.
__device__ __forceinline__ uint32_t box_muller(uint32_t f, float shift, float two)
{
    const float a = __uint_as_float((uint32_t)__builtin_amdgcn_mov_dpp((int)f, kDppPairFirst, 0xf, 0xf, true));
    const float b = __uint_as_float((uint32_t)__builtin_amdgcn_mov_dpp((int)f, kDppPairSecond, 0xf, 0xf, true));
    const float r = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(two - a));
    return __float_as_uint(r * __builtin_amdgcn_sinf(b + shift));
}

// Output stores go through a buffer resource covering exactly the round's
// cnt outputs: the hardware range check drops the stores of slots k >= cnt,
// so the store needs no branch (a branch lets the compiler sink the
// tempering loads behind it) and no 64-bit address arithmetic per lane.
// Word 3 is the gfx9-family default (32-bit data format). The stores are
// plain (cache policy 0): over the output layouts of batched plans a
// store-only kernel measured the nontemporal hint 3-5 % slower with one
// stream per workgroup and 42 % slower with one per wavefront.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kStorePolicy = 0;

// The window is the same for every lane of a wavefront; readfirstlane keeps
// the descriptor in scalar registers (a descriptor in vector registers makes
// every store a loop over the lanes' distinct descriptors).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_window(gu32 *p, uint32_t cnt)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    // readfirstlane returns int: take each half as uint32_t, so the low half
    // is zero-extended (sign extension would corrupt the address)
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    gu32 *q = reinterpret_cast<gu32 *>(((uint64_t)hi << 32) | lo);
    const uint32_t bytes = __builtin_amdgcn_readfirstlane(cnt * 4u);
    return __builtin_amdgcn_make_buffer_rsrc(static_cast<void *>(q), 0, (int)bytes, kBufferWord3);
}

// The recursion table rec[u & 0xf], evaluated one of two ways:
//   lookup (BASIS = false): a read of the 16-word table in LDS (3 vector
//       instructions per step, but the read sits on the round's chain);
//   basis  (BASIS = true): the table is F2-linear (the library rejects any
//       other), so rec[u & 0xf] is the XOR of rec[1 << b] over the set bits
//       b < 4 of u -- four sign-extended bit masks and four 3-input bit
//       operations against basis words in scalar registers (8 instructions,
//       no lookup on the chain).
// Which is faster depends on the launch (measured on gfx950: the lookup for
// batches of like generators filling every CU and for a single generator,
// the basis form for a mixed-period batch whose workgroups are wider than
// its smallest items' rounds); the launch shape chooses.
struct RecTable {
    const uint32_t *lds;          // rec[0..16) in LDS
    uint32_t b0, b1, b2, b3;      // rec[1], rec[2], rec[4], rec[8]
};

// x ^ (all-ones if bit b of u is set, else 0) & r, as one 3-input bit op
// (truth table 0x78 = a ^ (b & c) over the operand order x, mask, r).
template <int B>
__device__ __forceinline__ uint32_t xor_if_bit(uint32_t x, uint32_t u, uint32_t r)
{
    const uint32_t m = (uint32_t)__builtin_amdgcn_sbfe((int)u, B, 1);
    return __builtin_amdgcn_bitop3_b32(x, m, r, (uint8_t)0x78);
}

// u ^ rec[u & 0xf]
template <bool BASIS>
__device__ __forceinline__ uint32_t add_rec(uint32_t u, const RecTable &rt)
{
    if constexpr (BASIS) {
        uint32_t x = xor_if_bit<0>(u, u, rt.b0);
        x = xor_if_bit<1>(x, u, rt.b1);
        x = xor_if_bit<2>(x, u, rt.b2);
        return xor_if_bit<3>(x, u, rt.b3);
    } else {
        return u ^ rt.lds[u & 0xfu];
    }
}

// One round: SPL step slots per lane, slot c of lane `lane` is step
// k = lane + c*T of the round (T lanes). Xb points at x_{i0}; otb is the
// 16-word output table in LDS (16 distinct words in 16 banks: no conflicts).
template <int KIND, int SPL, bool BASIS>
__device__ __forceinline__ void round_steps(uint32_t *__restrict__ Xb, const RecTable &rt,
                                            const uint32_t *__restrict__ otb, uint32_t N, uint32_t M,
                                            uint32_t sh1, uint32_t sh2, uint32_t mask, uint32_t lane,
                                            uint32_t T, uint32_t cnt, gu32 *__restrict__ ob, float two)
{
    uint32_t xi[SPL], xi1[SPL], xt[SPL], xm[SPL];
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
        const uint32_t *xp = Xb + lane + c * T;
        xi[c] = xp[0];
        xi1[c] = xp[1];
        xt[c] = xp[M - 1];
        xm[c] = xp[M];
    }
    uint32_t x[SPL], tv[SPL];
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
        uint32_t s = xt[c] ^ (xt[c] >> 16);
        s ^= s >> 8;
        tv[c] = otb[s & 0xf];
    }
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
        const uint32_t a = xi1[c] ^ (xi[c] & mask);
        // u = a ^ (a << sh1) ^ (x_{i+M} >> sh2) as one 3-input XOR (truth table 0x96)
        const uint32_t u = __builtin_amdgcn_bitop3_b32(a << sh1, xm[c] >> sh2, a, (uint8_t)0x96);
        x[c] = add_rec<BASIS>(u, rt);
        Xb[N + lane + c * T] = x[c];
    }
    const __amdgpu_buffer_rsrc_t rsrc = out_window(ob, cnt);
    // angle offset of the normal kind: b - 1 (sine, odd lanes), b - 3/4 (cosine, even lanes)
    const float shift = (lane & 1u) ? -1.0f : -0.75f;
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
        const uint32_t k = lane + c * T;
        uint32_t o = output_word<KIND>(x[c], tv[c]);
        if constexpr (KIND == kKindNormal)
            o = box_muller(o, shift, two);   // steps k and k^1 are lanes lane and lane^1 (T is even)
        __builtin_amdgcn_raw_buffer_store_b32(o, rsrc, (int)(k * 4u), 0, kStorePolicy);
    }
}

// Rounds of one stream. All full rounds (cnt = W) run in runs between two
// compactions of the window, each run a tight 32-bit loop; the last,
// partial round (n mod W steps) follows. Loop control is scalar and
// per-round scalar work is kept to a few instructions, because in the group
// form every wavefront repeats it. WAVE: one wavefront, no barriers (LDS
// operations of a wavefront complete in order).
template <int KIND, int SPL, bool WAVE, bool BASIS>
__device__ __forceinline__ void run_stream(uint32_t *__restrict__ X, const RecTable &rt,
                                           const uint32_t *__restrict__ otb, uint32_t N, uint32_t M,
                                           uint32_t sh1, uint32_t sh2, uint32_t mask, uint32_t W,
                                           uint32_t L, uint64_t n, gu32 *__restrict__ out,
                                           uint32_t *__restrict__ state, uint32_t lane, uint32_t T)
{
    const uint32_t span = T * SPL;   // slots written per round
    // 2.0 in a vector register (normal kind), so that 2 - a can read a through DPP
    float two = 2.0f;
    if constexpr (KIND == kKindNormal)
        asm("v_mov_b32 %0, 2.0" : "=v"(two));
    uint64_t full = n / W;
    const uint32_t rem = (uint32_t)(n - full * W);
    uint32_t base = 0;
    gu32 *ob = out;
    while (full > 0) {
        if (base + N + span > L) {
            // base > L - N - span >= N: source and destination are disjoint
            for (uint32_t k = lane; k < N; k += T)
                X[k] = X[base + k];
            if (!WAVE)
                __syncthreads();
            base = 0;
        }
        // rounds that fit before the window must be compacted again
        const uint32_t room = (L - N - span - base) / W + 1;
        const uint32_t k = full < room ? (uint32_t)full : room;
        for (uint32_t j = 0; j < k; ++j) {
            round_steps<KIND, SPL, BASIS>(X + base, rt, otb, N, M, sh1, sh2, mask, lane, T, W, ob, two);
            if (!WAVE)
                __syncthreads();
            base += W;
            ob += W;
        }
        full -= k;
    }
    if (rem > 0) {
        if (base + N + span > L) {
            for (uint32_t k = lane; k < N; k += T)
                X[k] = X[base + k];
            if (!WAVE)
                __syncthreads();
            base = 0;
        }
        round_steps<KIND, SPL, BASIS>(X + base, rt, otb, N, M, sh1, sh2, mask, lane, T, rem, ob, two);
        if (!WAVE)
            __syncthreads();
        base += rem;
    }
    // x_n .. x_{n+N-1} back to HBM (section 8: the next call continues)
    if (state != nullptr)
        for (uint32_t k = lane; k < N; k += T)
            state[k] = X[base + k];
}

// ---------------------------------------------------------------------------
// The generation kernel. Two forms share the round code:
//   group (WAVE = false): the whole workgroup serves one generator; T lanes
//       take steps k = lane + c*T (c < spl) of each round, with a barrier
//       between rounds.
//   wave  (WAVE = true): each wavefront serves its own generator with its own
//       LDS window; steps k = lane + 64c. LDS operations of one wavefront
//       complete in issue order, so a round's reads see the previous round's
//       writes without a barrier or an LDS wait; the spl independent steps
//       per lane hide the LDS latency instead.
// Work comes from one item passed by value (grid of one), from item i for
// unit i, or -- persistent form -- from a queue in `counters`, in the order
// the host sorted the items (longest critical path first).
// LDS per unit: [0,16) recursion table, [16,32) output table, [32] queue
// slot, then the window X of L words.
// ---------------------------------------------------------------------------

template <int KIND, bool WAVE, bool BASIS>
__device__ __forceinline__ void run_item(uint32_t spl, uint32_t *X, const RecTable &rt, const uint32_t *otb,
                                         const GenRecord &g, uint32_t W, uint32_t L, uint64_t n, gu32 *out,
                                         uint32_t *state, uint32_t lane, uint32_t T)
{
#define MTGP_RUN(S) \
    run_stream<KIND, S, WAVE, BASIS>(X, rt, otb, g.N, g.M, g.sh1, g.sh2, g.mask, W, L, n, out, state, lane, T)
    if (WAVE) {
        switch (spl) {
        case 1: MTGP_RUN(1); break;
        case 2: MTGP_RUN(2); break;
        case 4: MTGP_RUN(4); break;
        case 6: MTGP_RUN(6); break;
        case 8: MTGP_RUN(8); break;
        case 12: MTGP_RUN(12); break;
        default: MTGP_RUN(16); break;
        }
    } else {
        switch (spl) {
        case 1: MTGP_RUN(1); break;
        case 2: MTGP_RUN(2); break;
        default: MTGP_RUN(4); break;
        }
    }
#undef MTGP_RUN
}

template <bool WAVE, bool BASIS>
__global__ __launch_bounds__(1024) void mtgp_kernel(const GenRecord *__restrict__ recs, uint32_t *__restrict__ states,
                                                    const WorkItem *__restrict__ items, uint32_t nitems,
                                                    uint32_t *counters, WorkItem single, uint32_t L)
{
    extern __shared__ uint32_t smem[];
    const uint32_t lane = WAVE ? (threadIdx.x & 63u) : threadIdx.x;
    const uint32_t T = WAVE ? 64u : blockDim.x;
    // the unit index is the same in every lane of a wavefront; readfirstlane
    // tells the compiler so, keeping the unit's item, window and output
    // descriptor in scalar registers (else each buffer store becomes a loop
    // over the lanes' descriptors)
    const uint32_t unit = WAVE ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0u;
    const uint32_t units = WAVE ? (blockDim.x >> 6) : 1u;
    uint32_t *unit_lds = smem + unit * (kTableWords + L);
    uint32_t *rtb = unit_lds;
    uint32_t *otb = unit_lds + 16;
    uint32_t *qslot = unit_lds + 32;
    uint32_t *X = unit_lds + kTableWords;

    for (uint32_t iter = 0;; ++iter) {
        WorkItem it;
        if (items == nullptr) {                 // one item passed by value, one unit
            if (iter > 0 || blockIdx.x > 0 || unit > 0)
                break;
            it = single;
        } else if (counters == nullptr) {       // item i in unit i
            const uint32_t w = blockIdx.x * units + unit;
            if (iter > 0 || w >= nitems)
                break;
            it = items[w];
        } else {                                // persistent: pop from the queue
            // (units that start late -- a grid larger than what fits at once
            // -- then take the next item in order, which keeps the longest-
            // first order; assigning item w to unit w up front did not)
            uint32_t q;
            if (WAVE) {
                q = 0;
                if (lane == 0)
                    q = atomicAdd(&counters[0], 1u);
                q = __builtin_amdgcn_readfirstlane(q);
            } else {
                if (lane == 0)
                    qslot[0] = atomicAdd(&counters[0], 1u);
                __syncthreads();
                q = __builtin_amdgcn_readfirstlane(qslot[0]);
                __syncthreads();
            }
            if (q >= nitems)
                break;
            it = items[q];
        }
        const uint32_t gen = __builtin_amdgcn_readfirstlane(it.gen);
        const uint32_t flags = __builtin_amdgcn_readfirstlane((uint32_t)it.kind);
        const uint32_t kind = flags & 0xffu;
        const uint32_t spl = __builtin_amdgcn_readfirstlane((uint32_t)it.spl);
        const GenRecord &g = recs[gen];
        const uint32_t N = g.N, M = g.M;
        uint32_t *slot = states + g.state_off;
        const uint32_t *from = it.src ? reinterpret_cast<const uint32_t *>(it.src) : slot;
        uint32_t *state = (flags & kKeepState)    ? nullptr
                          : (flags & kStateToSrc) ? const_cast<uint32_t *>(from)
                                                  : slot;
        uint32_t W = (N - M) < T * spl ? (N - M) : T * spl;
        if (kind == kKindNormal)
            W &= ~1u;   // rounds of whole pairs (the host requires N - M >= 2 for this kind)
        if (W == 0)
            W = 1;      // never reached through the library; keeps the loop bounds finite

        for (uint32_t k = lane; k < N; k += T)
            X[k] = from[k];
        if (lane < 16) {
            rtb[lane] = g.rec[lane];
            otb[lane] = kind == 0 ? g.tmp[lane] : g.flt[lane];
        }
        const RecTable rt = {rtb, g.rec[1], g.rec[2], g.rec[4], g.rec[8]};
        if (!WAVE)
            __syncthreads();

        gu32 *out = reinterpret_cast<gu32 *>(it.out);
        if (kind == kKindRaw) {
            // the start words first, then the new words
            for (uint32_t k = lane; k < N; k += T)
                out[k] = X[k];
            out += N;
        }
        if (kind == kKindU32)
            run_item<kKindU32, WAVE, BASIS>(spl, X, rt, otb, g, W, L, it.n, out, state, lane, T);
        else if (kind == kKindF12)
            run_item<kKindF12, WAVE, BASIS>(spl, X, rt, otb, g, W, L, it.n, out, state, lane, T);
        else if (kind == kKindF01)
            run_item<kKindF01, WAVE, BASIS>(spl, X, rt, otb, g, W, L, it.n, out, state, lane, T);
        else if (kind == kKindNormal)
            run_item<kKindNormal, WAVE, BASIS>(spl, X, rt, otb, g, W, L, it.n, out, state, lane, T);
        else
            run_item<kKindRaw, WAVE, BASIS>(spl, X, rt, otb, g, W, L, it.n, out, state, lane, T);
        if (!WAVE)
            __syncthreads();   // the next item overwrites the window and tables
    }

    // Queue reset by the last unit to finish. Each unit's last pop returned
    // its value (the loop tested it) before this increment is issued, so all
    // pops are performed once the count reaches the total; no fence is
    // needed (a device-scope fence here compiles to an L2 write-back and
    // invalidate per unit, which slowed the launch's tail measurably). The
    // outputs need none either: the end of the kernel makes them visible.
    if (items != nullptr && counters != nullptr && lane == 0) {
        const uint32_t done = atomicAdd(&counters[1], 1u);
        if (done == gridDim.x * units - 1) {    // every pop has returned: reset for the next launch
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// Chunked wavefront form (kModeChunk). One wavefront runs one work item at a
// time, with no barrier. The stream is cut into chunks of 64 consecutive
// steps, one step per lane. Step j reads x_j, x_{j+1}, x_{j+M-1} and
// x_{j+M}; the newest of them was written by step j - (N - M). So when
// N - M >= 192, chunk q+2 depends only on chunks up to q-1, and the loop keeps
// three chunks in flight: it issues the LDS reads of chunk q+2, computes chunk
// q+1 up to its table lookups, and finishes chunk q (new word back to LDS,
// output converted and stored). LDS operations of one wavefront complete in
// issue order, so the reads of chunk q+3, issued after chunk q's write, see
// it. This is section 3.2's round parallelism with the N - M independent steps
// taken 64 at a time in a software pipeline instead of all at once behind a
// barrier.
//
// The state lives in a ring of L words (L a power of two, L >= N + 64): the
// new word x_{N+j} sits in slot j mod L, the start words x_k (k < N) in slots
// L - N + k, and every word is stored twice, at its slot and L slots on (two
// LDS writes). The words step j reads, x_j .. x_{j+M}, are then found at
// slots (j mod L) + L - N .. (j mod L) + L - N + M, all below 2L: the reads
// never wrap and no compaction copy is needed. (Writing the second copy only
// for the chunks that need it takes a branch per chunk, after which the
// compiler waits for every outstanding LDS operation and the pipeline
// drains.) LDS per wavefront: 2L ring words at a multiple of 2L words; after
// all rings, each wavefront's 16-word recursion table and 16-word output
// table, each at a multiple of 64 bytes, so a lookup's address is
// (4 index) | table base.
// ---------------------------------------------------------------------------

typedef __attribute__((address_space(3))) uint32_t lds_word;

// HBM words through global-address-space pointers: generic (flat) accesses
// also count on the LDS counter, and with one possibly outstanding the
// compiler can only wait for all LDS operations
typedef __attribute__((address_space(1))) uint32_t hbm_word;

__device__ __forceinline__ uint32_t hbm_get(const uint32_t *p, uint32_t k)
{
    return ((const hbm_word *)p)[k];
}

__device__ __forceinline__ void hbm_put(uint32_t *p, uint32_t k, uint32_t v)
{
    ((hbm_word *)p)[k] = v;
}

// s_waitcnt immediate for lgkmcnt(0) with the other counters unconstrained
// (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitLgkm0 = 0xc07f;

__device__ __forceinline__ uint32_t lds_get(uint32_t byte)
{
    return *(lds_word *)(uintptr_t)byte;
}

__device__ __forceinline__ void lds_put(uint32_t byte, uint32_t v)
{
    *(lds_word *)(uintptr_t)byte = v;
}

// Words of one chunk read from the ring: x_j, x_{j+1}, x_{j+M-1}, x_{j+M}.
struct ChunkIn {
    uint32_t a, b, c, d;
};

// A chunk after the recursion up to the table lookups: u, rec[u & 0xf] and
// the output-table entry of the tempering index.
struct ChunkMid {
    uint32_t u, r, t;
};

template <int KIND, uint32_t L, uint32_t RA, uint32_t CA>
__device__ __forceinline__ void chunk_stream(uint32_t ringb, uint32_t rtab, uint32_t otab, uint32_t N, uint32_t M,
                                             uint32_t sh1, uint32_t sh2, uint32_t mask, uint64_t n, gu32 *out,
                                             uint32_t *state, const uint32_t *from, uint32_t lane)
{
    // 2.0 in a vector register (normal kind), so that 2 - a can read a through DPP
    float two = 2.0f;
    if constexpr (KIND == kKindNormal)
        asm("v_mov_b32 %0, 2.0" : "=v"(two));
    // Ring layout: x_{N+j} sits at slot j mod L and again at slot j mod L + L,
    // the start words x_k (k < N) at slots L - N + k and 2L - N + k. The slots
    // a chunk writes are then aligned to the chunk, and the words it reads sit
    // L - N slots past them, never past slot 2L: inside a block of eight chunks
    // (512 slots, one part of a turn of the ring) every LDS address is a
    // register set once per block plus an immediate offset.
    for (uint32_t k = lane; k < N; k += 64) {
        const uint32_t v = hbm_get(from, k);
        lds_put(ringb + 4u * (L - N + k), v);
        lds_put(ringb + 4u * (2u * L - N + k), v);
    }
    const uint32_t rA = ringb + 4u * (L - N + lane);   // slot of x_j for the step j = lane
    const uint32_t rC = rA + 4u * (M - 1u);            // slot of x_{j+M-1}
    const uint32_t wA = ringb + 4u * lane;             // slot of x_{N+j}
    const float shift = (lane & 1u) ? -1.0f : -0.75f;  // normal kind: angle offsets of cos and sin lanes
    // byte offset of chunk q's slots from the ring base
    auto ring_off = [](uint64_t q) { return 4u * ((64u * (uint32_t)q) & (L - 1u)); };

    auto reads = [&](uint32_t pa, uint32_t pc) {
        ChunkIn c;
        c.a = lds_get(pa);
        c.b = lds_get(pa + 4u);
        c.c = lds_get(pc);
        c.d = lds_get(pc + 4u);
        return c;
    };
    auto compute = [&](const ChunkIn &c) {
        ChunkMid m;
        const uint32_t a = __builtin_amdgcn_bitop3_b32(c.b, c.a, mask, (uint8_t)0x78);   // x_{j+1} ^ (x_j & mask)
        m.u = __builtin_amdgcn_bitop3_b32(a << sh1, c.d >> sh2, a, (uint8_t)0x96);
        m.r = lds_get(((m.u << 2) & 0x3cu) | rtab);
        if constexpr (KIND != kKindRaw) {
            // only the low four bits of the index count, so each fold is one
            // XOR with a halfword or byte operand select (the compiler finds
            // the first and not the second)
            const uint32_t h = c.c ^ (c.c >> 16);
            uint32_t t;
            asm("v_xor_b32_sdwa %0, %1, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
                : "=v"(t)
                : "v"(h));
            m.t = lds_get(((t << 2) & 0x3cu) | otab);
        } else {
            m.t = 0;
        }
        return m;
    };
    auto finish = [&](uint32_t w, const ChunkMid &m, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
        const uint32_t x = m.u ^ m.r;
        lds_put(w, x);
        lds_put(w + 4u * L, x);
        uint32_t o = output_word<KIND>(x, m.t);
        if constexpr (KIND == kKindNormal)
            o = box_muller(o, shift, two);   // steps 2i and 2i+1 are lanes 2l and 2l+1 of one chunk
        __builtin_amdgcn_raw_buffer_store_b32(o, rs, (int)(4u * lane + off), 0, kStorePolicy);
    };

    const uint64_t Q = (n + 63) / 64;
    // no scalar load may be outstanding inside the loop: scalar loads share
    // the LDS counter but complete out of order, and with one pending the
    // compiler can only wait for all LDS operations instead of the oldest
    __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
    // iteration q issues the reads of chunk q + RA, computes chunk q + CA up
    // to its table lookups and finishes chunk q; reads wait RA - CA
    // iterations for their data, lookups CA iterations
    ChunkIn in[RA];
    ChunkMid mid[CA];
#pragma unroll
    for (uint32_t k = 0; k < RA; k++)
        in[k] = reads(rA + 256u * k, rC + 256u * k);
#pragma unroll
    for (uint32_t k = 0; k < CA; k++) {
        mid[k] = compute(in[0]);
#pragma unroll
        for (uint32_t r = 0; r + 1 < RA; r++)
            in[r] = in[r + 1];
        in[RA - 1] = reads(rA + 256u * (RA + k), rC + 256u * (RA + k));
    }
    // one iteration: the reads of a later chunk at (pa, pc), the computation
    // of the next chunk up to its lookups, and this chunk's words to slot w
    auto step = [&](uint32_t pa, uint32_t pc, uint32_t w, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
        // the stages stay in this order: left to itself, the scheduler
        // moves each chunk's computation next to its reads, and the
        // pipeline becomes a wait for every read
        const ChunkIn fresh = reads(pa, pc);
        __builtin_amdgcn_sched_barrier(0);
        const ChunkMid m = compute(in[0]);
        __builtin_amdgcn_sched_barrier(0);
        finish(w, mid[0], rs, off);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (uint32_t r = 0; r + 1 < RA; r++)
            in[r] = in[r + 1];
        in[RA - 1] = fresh;
#pragma unroll
        for (uint32_t r = 0; r + 1 < CA; r++)
            mid[r] = mid[r + 1];
        mid[CA - 1] = m;
    };
    constexpr uint32_t F = CA + RA;   // the fresh reads are F chunks ahead
    static_assert(F < 8, "read-ahead within one block");
    uint64_t q = 0;
    // blocks of eight chunks: one output window (the range check drops the
    // stores of steps >= n), stores at immediate offsets; the block's slots
    // start at a0 and the next block's at a1 (the same for a 512-slot ring)
    uint32_t a0 = 0;
    for (; q + 8 <= Q; q += 8) {
        const uint32_t a1 = L == 512 ? 0u : (a0 + 2048u) & (4u * L - 1u);
        const uint32_t pa0 = rA + a0, pc0 = rC + a0, pa1 = rA + a1, pc1 = rC + a1, w0 = wA + a0;
        const __amdgpu_buffer_rsrc_t rs = out_window(out + 64 * q, (uint32_t)std::min<uint64_t>(n - 64 * q, 512));
#pragma unroll
        for (uint32_t j = 0; j < 8; j++) {
            const uint32_t f = j + F;
            if (f < 8)
                step(pa0 + 256u * f, pc0 + 256u * f, w0 + 256u * j, rs, 256u * j);
            else
                step(pa1 + 256u * (f - 8u), pc1 + 256u * (f - 8u), w0 + 256u * j, rs, 256u * j);
        }
        a0 = a1;
    }
    for (; q < Q; q++) {
        const uint32_t af = ring_off(q + F);
        step(rA + af, rC + af, wA + ring_off(q), out_window(out + 64 * q, (uint32_t)std::min<uint64_t>(n - 64 * q, 64)),
             0);
    }
    // x_n .. x_{n+N-1} back to HBM (section 8: the next call continues)
    if (state != nullptr)
        for (uint32_t k = lane; k < N; k += 64)
            hbm_put(state, k, lds_get(ringb + 4u * (((uint32_t)n + k + L - N) & (L - 1u))));
}

// One item in a ring of L words, dispatched on its output kind.
template <uint32_t L, uint32_t RA, uint32_t CA>
__device__ __forceinline__ void chunk_kind(uint32_t kind, uint32_t ringb, uint32_t rtab, uint32_t otab, uint32_t N,
                                           uint32_t M, const GenRecord &g, uint64_t n, gu32 *out, uint32_t *state,
                                           const uint32_t *from, uint32_t lane)
{
#define MTGP_CHUNK(K) chunk_stream<K, L, RA, CA>(ringb, rtab, otab, N, M, g.sh1, g.sh2, g.mask, n, out, state, from, lane)
    if (kind == kKindU32)
        MTGP_CHUNK(kKindU32);
    else if (kind == kKindF12)
        MTGP_CHUNK(kKindF12);
    else if (kind == kKindF01)
        MTGP_CHUNK(kKindF01);
    else if (kind == kKindNormal)
        MTGP_CHUNK(kKindNormal);
    else
        MTGP_CHUNK(kKindRaw);
#undef MTGP_CHUNK
}

// The chunked form's kernel: each wavefront pops work items like the wave
// form (persistent queue, one item passed by value, or item i for unit i).
template <uint32_t L, uint32_t RA, uint32_t CA>
__global__ __launch_bounds__(1024) void mtgp_chunk_kernel(const GenRecord *__restrict__ recs,
                                                          uint32_t *__restrict__ states,
                                                          const WorkItem *__restrict__ items, uint32_t nitems,
                                                          uint32_t *counters, WorkItem single)
{
    extern __shared__ uint32_t smem[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t unit = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t units = blockDim.x >> 6;
    // dynamic LDS starts at byte 0 in this kernel (it declares no static
    // LDS), so ring bases are multiples of 8L bytes
    const uint32_t base = (uint32_t)(uintptr_t)(lds_word *)smem;
    const uint32_t ringb = base + unit * 8u * L;
    const uint32_t rtab = base + units * 8u * L + unit * 128u;
    const uint32_t otab = rtab + 64u;

    for (uint32_t iter = 0;; ++iter) {
        WorkItem it;
        if (items == nullptr) {
            if (iter > 0 || blockIdx.x > 0 || unit > 0)
                break;
            it = single;
        } else if (counters == nullptr) {
            const uint32_t w = blockIdx.x * units + unit;
            if (iter > 0 || w >= nitems)
                break;
            it = items[w];
        } else {
            uint32_t q = 0;
            if (lane == 0)
                q = atomicAdd(&counters[0], 1u);
            q = __builtin_amdgcn_readfirstlane(q);
            if (q >= nitems)
                break;
            it = items[q];
        }
        const uint32_t gen = __builtin_amdgcn_readfirstlane(it.gen);
        const uint32_t flags = __builtin_amdgcn_readfirstlane((uint32_t)it.kind);
        const uint32_t kind = flags & 0xffu;
        const GenRecord &g = recs[gen];
        const uint32_t N = g.N, M = g.M;
        uint32_t *slot = states + g.state_off;
        const uint32_t *from = it.src ? reinterpret_cast<const uint32_t *>(it.src) : slot;
        uint32_t *state = (flags & kKeepState)    ? nullptr
                          : (flags & kStateToSrc) ? const_cast<uint32_t *>(from)
                                                  : slot;
        if (lane < 16) {
            lds_put(rtab + 4u * lane, g.rec[lane]);
            lds_put(otab + 4u * lane, kind == kKindU32 ? g.tmp[lane] : g.flt[lane]);
        }
        gu32 *out = reinterpret_cast<gu32 *>(it.out);
        if (kind == kKindRaw) {
            // the start words first, then the new words
            for (uint32_t k = lane; k < N; k += 64)
                hbm_put(out, k, hbm_get(from, k));
            out += N;
        }
        // each item runs in the ring its own state needs (the wavefront's LDS
        // region is sized for the launch's largest): with a 512-word ring a
        // block of eight chunks is one turn of the ring, and the compiler
        // keeps every LDS address of the block in registers
        const uint32_t LI = chunk_ring_words(N);
        if (LI <= 512 || L == 512)
            chunk_kind<(L < 512 ? L : 512), RA, CA>(kind, ringb, rtab, otab, N, M, g, it.n, out, state, from, lane);
        else if (LI <= 1024 || L == 1024)
            chunk_kind<(L < 1024 ? L : 1024), RA, CA>(kind, ringb, rtab, otab, N, M, g, it.n, out, state, from, lane);
        else if (LI <= 2048 || L == 2048)
            chunk_kind<(L < 2048 ? L : 2048), RA, CA>(kind, ringb, rtab, otab, N, M, g, it.n, out, state, from, lane);
        else
            chunk_kind<L, RA, CA>(kind, ringb, rtab, otab, N, M, g, it.n, out, state, from, lane);
    }
    // queue reset by the last unit to finish (as in mtgp_kernel)
    if (items != nullptr && counters != nullptr && lane == 0) {
        const uint32_t done = atomicAdd(&counters[1], 1u);
        if (done == gridDim.x * units - 1) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
}

hipError_t launch_generate(const GenRecord *recs, uint32_t *states, const WorkItem *items, uint32_t nitems,
                           uint32_t *counters, const WorkItem &single, const LaunchShape &shape,
                           hipStream_t stream)
{
    const dim3 grid(shape.grid), block(shape.threads);
    const uint32_t L = (uint32_t)shape.lds_words;
    const uint32_t units = shape.mode == kModeGroup ? 1u : (uint32_t)(shape.threads / 64);
    if (shape.mode == kModeChunk) {
        const size_t lds_c = (size_t)(shape.threads / 64) * (2u * L + 32u) * sizeof(uint32_t);
#define MTGP_LAUNCH_CHUNK(LL, RA, CA) \
    hipLaunchKernelGGL((mtgp_chunk_kernel<LL, RA, CA>), grid, block, lds_c, stream, recs, states, items, nitems, \
                       counters, single)
#define MTGP_LAUNCH_CHUNK_L(LL) \
    if (shape.spl == 2) MTGP_LAUNCH_CHUNK(LL, 2, 1); \
    else MTGP_LAUNCH_CHUNK(LL, 1, 1);
        switch (L) {
        case 512: MTGP_LAUNCH_CHUNK_L(512); break;
        case 1024: MTGP_LAUNCH_CHUNK_L(1024); break;
        case 2048: MTGP_LAUNCH_CHUNK_L(2048); break;
        case 4096: MTGP_LAUNCH_CHUNK_L(4096); break;
        default: return hipErrorInvalidValue;
        }
#undef MTGP_LAUNCH_CHUNK_L
#undef MTGP_LAUNCH_CHUNK
        return hipGetLastError();
    }
    const size_t lds = (size_t)units * (kTableWords + L) * sizeof(uint32_t);
#define MTGP_LAUNCH(W, B) \
    hipLaunchKernelGGL((mtgp_kernel<W, B>), grid, block, lds, stream, recs, states, items, nitems, counters, single, L)
    if (shape.mode == kModeGroup) {
        if (shape.rec_basis)
            MTGP_LAUNCH(false, true);
        else
            MTGP_LAUNCH(false, false);
    } else {
        if (shape.rec_basis)
            MTGP_LAUNCH(true, true);
        else
            MTGP_LAUNCH(true, false);
    }
#undef MTGP_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Jump correlation: a start state F^J S = h(F) S as the XOR of the states
// S, F S, F^2 S, ... selected by the coefficients of h = x^J mod psi (psi an
// annihilating polynomial of S), i.e. out[w] = XOR_{i: h_i = 1} raw[i + w].
//
// One workgroup of G P wavefronts per jump. Lane l of wavefront g owns the R
// consecutive words w0 .. w0+R-1 (w0 = 64 R g + R l) and slides a 2R-word
// window (lo, hi) = raw[i + w0 .. i + w0 + 2R) over the bits of h: per block
// of R bits it XORs, for each set bit t (a uniform scalar test), the window
// words t .. t+R-1 into its sums, so a clear bit costs no vector work. The
// window then moves on by R words: the new lo is the old hi, and the new hi is
// the next lane's new lo, taken across lanes with a wave-wide DPP shift; only
// the top lane's R words come from LDS, as a broadcast read. The P wavefronts
// of a word group split the bits of h and add their partial sums through LDS
// at the end. The block bits come from h's 64-bit words, staged in LDS beside
// raw and read one iteration ahead.
// ---------------------------------------------------------------------------

constexpr int kDppWaveShl1 = 0x130;   // DPP control: lane k reads lane k + 1; lane 63 keeps `old`

// One block: R bits hb of h over the window (lo, hi); then nx = the next hi,
// shifted in from lane + 1, with the top lane's words read from top[].
template <uint32_t R>
__device__ __forceinline__ void jump_block(uint32_t (&acc)[R], const uint32_t (&lo)[R], const uint32_t (&hi)[R],
                                           uint32_t (&nx)[R], const uint32_t *top, uint32_t hb)
{
    uint32_t ext[R];
#pragma unroll
    for (uint32_t r = 0; r < R; r++)
        ext[r] = top[r];   // same address in every lane: an LDS broadcast
#pragma unroll
    for (uint32_t t = 0; t < R; t++) {
        if ((hb >> t) & 1u) {   // uniform: a clear bit costs no vector work
            // an empty volatile asm keeps the compiler from turning the
            // branch into XORs and selects for every bit
            asm volatile("");
#pragma unroll
            for (uint32_t r = 0; r < R; r++)
                acc[r] ^= (t + r < R) ? lo[t + r] : hi[t + r - R];
        }
    }
#pragma unroll
    for (uint32_t r = 0; r < R; r++)
        nx[r] = (uint32_t)__builtin_amdgcn_update_dpp((int)ext[r], (int)hi[r], kDppWaveShl1, 0xf, 0xf, false);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

template <uint32_t R>
__global__ __launch_bounds__(1024) void mtgp_jump_kernel(const JumpItem *__restrict__ items)
{
    extern __shared__ uint32_t Xs[];
    const JumpItem it = items[blockIdx.x];
    constexpr uint32_t W = 64 * R;          // words per wavefront
    constexpr uint32_t STEP = 4 * R;        // bits (and raw words) per iteration
    const JumpShape sh = jump_shape(it.N);  // sh.R == R
    const uint32_t N = it.N, D = it.D;
    // P wavefronts per word group: the launch sizes the workgroup to G * P wavefronts
    const uint32_t G = sh.G, P = (blockDim.x >> 6) / sh.G, CI = sh.CI;
    const uint32_t raw_words = 4 * R * CI + G * W + 6 * R;
    uint64_t *Ps = reinterpret_cast<uint64_t *>(Xs + (raw_words + 1) / 2 * 2);
    const uint32_t *raw = reinterpret_cast<const uint32_t *>(it.raw);
    const uint64_t *poly = reinterpret_cast<const uint64_t *>(it.poly);
    uint32_t *out = reinterpret_cast<uint32_t *>(it.out);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const bool active = wave < G * P;
    const uint32_t grp = wave % G;
    const uint32_t part = wave / G;
    const uint32_t w0 = grp * W + lane * R;
    const uint32_t wtop = (grp + 1) * W;            // first word past this wavefront's words
    const uint32_t iters = (D + STEP - 1) / STEP;   // 64-bit words of h

    uint32_t acc[R];
#pragma unroll
    for (uint32_t r = 0; r < R; r++)
        acc[r] = 0;

    for (uint32_t s0 = 0; s0 < iters; s0 += CI) {
        const uint32_t ci = iters - s0 < CI ? iters - s0 : CI;
        const uint32_t i0 = s0 * STEP;
        const uint32_t cnt = D - i0 < ci * STEP ? D - i0 : ci * STEP;
        for (uint32_t k = threadIdx.x; k < cnt + N - 1; k += blockDim.x)
            Xs[k] = raw[i0 + k];
        for (uint32_t k = threadIdx.x; k < ci; k += blockDim.x)
            Ps[k] = poly[s0 + k];
        __syncthreads();
        if (active) {
            // this wavefront's iterations of the stage: [q0, q1)
            const uint32_t per = (ci + P - 1) / P;
            const uint32_t q0 = part * per;
            const uint32_t q1 = q0 + per < ci ? q0 + per : ci;
            uint32_t A[R], B[R];
            if (q0 < q1) {
                uint32_t ext[R];
#pragma unroll
                for (uint32_t r = 0; r < R; r++) {
                    A[r] = Xs[q0 * STEP + w0 + r];
                    ext[r] = Xs[q0 * STEP + wtop + r];
                }
#pragma unroll
                for (uint32_t r = 0; r < R; r++)
                    B[r] = (uint32_t)__builtin_amdgcn_update_dpp((int)ext[r], (int)A[r], kDppWaveShl1, 0xf, 0xf,
                                                                 false);
            }
            uint64_t hw = q0 < q1 ? uniform64(Ps[q0]) : 0;
            for (uint32_t q = q0; q < q1; q++) {
                const uint64_t hn = q + 1 < q1 ? uniform64(Ps[q + 1]) : 0;
                // the top lane's next hi for block b is raw[i + (b + 2) R + wtop ..]
                const uint32_t *top = Xs + q * STEP + wtop;
                jump_block<R>(acc, A, B, A, top + 1 * R, (uint32_t)hw & 0xffffu);
                jump_block<R>(acc, B, A, B, top + 2 * R, (uint32_t)(hw >> 16) & 0xffffu);
                jump_block<R>(acc, A, B, A, top + 3 * R, (uint32_t)(hw >> 32) & 0xffffu);
                jump_block<R>(acc, B, A, B, top + 4 * R, (uint32_t)(hw >> 48));
                hw = hn;
            }
        }
        __syncthreads();
    }
    // partial sums of the P wavefronts of each word group, through LDS
    if (P > 1) {
        if (active && part > 0)
#pragma unroll
            for (uint32_t r = 0; r < R; r++)
                Xs[(part - 1) * (G * W) + w0 + r] = acc[r];
        __syncthreads();
        if (active && part == 0)
            for (uint32_t q = 1; q < P; q++)
#pragma unroll
                for (uint32_t r = 0; r < R; r++)
                    acc[r] ^= Xs[(q - 1) * (G * W) + w0 + r];
    }
    if (active && part == 0)
#pragma unroll
        for (uint32_t r = 0; r < R; r++)
            if (w0 + r < N)
                out[w0 + r] = acc[r];
}

template <uint32_t R>
hipError_t launch_jump_run(const JumpItem *items, uint32_t n, uint32_t threads, size_t lds, hipStream_t stream)
{
    hipLaunchKernelGGL(mtgp_jump_kernel<R>, dim3(n), dim3(threads), lds, stream, items);
    return hipGetLastError();
}

template <uint32_t R>
hipError_t launch_jump_width(uint32_t width, const JumpItem *items, uint32_t n, uint32_t threads, size_t lds,
                             hipStream_t stream)
{
    if constexpr (R > kJumpMaxR) {
        return hipErrorInvalidValue;
    } else {
        return width == R ? launch_jump_run<R>(items, n, threads, lds, stream)
                          : launch_jump_width<R + 1>(width, items, n, threads, lds, stream);
    }
}

hipError_t launch_jumps(const JumpItem *d_items, const JumpItem *h_items, uint32_t nitems, hipStream_t stream)
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    // one launch per run of items with the same lane width and word groups
    uint32_t k = 0;
    while (k < nitems) {
        const JumpShape s = jump_shape(h_items[k].N);
        uint32_t e = k;
        while (e < nitems && jump_shape(h_items[e].N).R == s.R && jump_shape(h_items[e].N).G == s.G)
            e++;
        // Each jump is a sequential pass over the bits of h split among P
        // wavefronts per word group; with few jumps per CU that pass is the
        // launch's latency, so P doubles (up to 16 wavefronts a workgroup)
        // until about 16 wavefronts per CU are busy.
        uint32_t P = s.P;
        while (s.G * P * 2 <= 16 && (uint64_t)(e - k) * s.G * P < 16ull * (uint64_t)cus)
            P *= 2;
        uint32_t words = 0;
        for (uint32_t i = k; i < e; i++) {
            const uint32_t own = jump_lds_words(h_items[i].N);
            const uint32_t sums = (P - 1) * s.G * 64 * s.R;   // partial sums of the extra wavefronts
            words = own > words ? own : words;
            words = sums > words ? sums : words;
        }
        const hipError_t err =
            launch_jump_width<kJumpMinR>(s.R, d_items + k, e - k, 64 * s.G * P, (size_t)words * 4u, stream);
        if (err != hipSuccess)
            return err;
        k = e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Fixed device scratch of the allocation-free batch call
// (mtgp_batch_generate_static): the queue counters in its first 256 bytes,
// then up to kStaticMaxItems work items. One copy per GPU, for the life of
// the process; every such call on a GPU uses that GPU's copy.
// ---------------------------------------------------------------------------

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        // the symbol's address on this device (host code must not pass the
        // array's name itself to a kernel: it stands for no device address)
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

__global__ void mtgp_zero_words(uint32_t *p, uint32_t n)
{
    for (uint32_t k = threadIdx.x; k < n; k += blockDim.x)
        p[k] = 0;
}

hipError_t launch_zero_words(uint32_t *p, uint32_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(mtgp_zero_words, dim3(1), dim3(64), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t opt_in_lds(size_t bytes)
{
    const int b = (int)bytes;
    const void *kernels[] = {reinterpret_cast<const void *>(&mtgp_kernel<false, false>),
                             reinterpret_cast<const void *>(&mtgp_kernel<false, true>),
                             reinterpret_cast<const void *>(&mtgp_kernel<true, false>),
                             reinterpret_cast<const void *>(&mtgp_kernel<true, true>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<512, 1, 1>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<512, 2, 1>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<1024, 1, 1>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<1024, 2, 1>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<2048, 1, 1>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<2048, 2, 1>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<4096, 1, 1>),
                             reinterpret_cast<const void *>(&mtgp_chunk_kernel<4096, 2, 1>)};
    for (const void *k : kernels) {
        const hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, b);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace mtgp_impl
