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
// Loads of a round are issued first, then both table lookups, then the
// writes, so a round costs two LDS round trips plus its barrier.
//
// Step k of a round is done by lane k mod T in pass k / T (T = workgroup
// size), so LDS reads and writes are unit-stride across a wavefront and the
// outputs of a pass are one contiguous, coalesced nontemporal store.
//
// Per step (section 3.6 and 3.7):
//   t = x_{i+1} ^ (x_i & mask);  t ^= t << sh1;  u = t ^ (x_{i+M} >> sh2)
//   x_{i+N} = u ^ rec[u & 0xf]
//   s = x_{i+M-1} ^ (x_{i+M-1} >> 16);  s ^= s >> 8
//   uint32:      o = x_{i+N} ^ tmp[s & 0xf]
//   float [1,2): o = (x_{i+N} >> 9) ^ flt[s & 0xf]       (section 6, eq. (C))
//   float [0,1): the [1,2) value minus 1.0f
#include "mtgp_internal.h"

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
    if constexpr (KIND == 0) {
        return x ^ tv;
    } else {
        const uint32_t b = (x >> 9) ^ tv;
        if constexpr (KIND == 1) {
            return b;
        } else {
            return __float_as_uint(__uint_as_float(b) - 1.0f);
        }
    }
}

// Output stores go through a buffer resource covering exactly the round's
// cnt outputs: the hardware range check drops the stores of slots k >= cnt,
// so the store needs no branch (a branch lets the compiler sink the
// tempering loads behind it) and no 64-bit address arithmetic per lane.
// Word 3 is the gfx9-family default (32-bit data format); cache policy 2 sets
// the nontemporal bit.
constexpr int kBufferWord3 = 0x00020000;
constexpr int kStoreNT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_window(gu32 *p, uint32_t cnt)
{
    return __builtin_amdgcn_make_buffer_rsrc(static_cast<void *>(p), 0, (int)(cnt * 4u), kBufferWord3);
}

// One round: SPL step slots per lane, slot c of lane `lane` is step
// k = lane + c*T of the round (T lanes). Xb points at x_{i0}.
template <int KIND, int SPL>
__device__ __forceinline__ void round_steps(uint32_t *__restrict__ Xb, const uint32_t *__restrict__ rec,
                                            const uint32_t *__restrict__ otb, uint32_t N, uint32_t M,
                                            uint32_t sh1, uint32_t sh2, uint32_t mask, uint32_t lane,
                                            uint32_t T, uint32_t cnt, gu32 *__restrict__ ob)
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
    uint32_t u[SPL], rv[SPL], tv[SPL];
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
        uint32_t a = xi1[c] ^ (xi[c] & mask);
        a ^= a << sh1;
        u[c] = a ^ (xm[c] >> sh2);
        uint32_t s = xt[c] ^ (xt[c] >> 16);
        s ^= s >> 8;
        rv[c] = rec[u[c] & 0xf];
        tv[c] = otb[s & 0xf];
    }
    const __amdgpu_buffer_rsrc_t rsrc = out_window(ob, cnt);
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
        const uint32_t k = lane + c * T;
        const uint32_t x = u[c] ^ rv[c];
        Xb[N + k] = x;
        __builtin_amdgcn_raw_buffer_store_b32(output_word<KIND>(x, tv[c]), rsrc, (int)(k * 4u), 0, kStoreNT);
    }
}

template <int KIND, int SPL>
__device__ __forceinline__ void run_stream(uint32_t *__restrict__ X, const uint32_t *__restrict__ rec,
                                           const uint32_t *__restrict__ otb, uint32_t N, uint32_t M,
                                           uint32_t sh1, uint32_t sh2, uint32_t mask, uint32_t W,
                                           uint32_t L, uint64_t n, gu32 *__restrict__ out,
                                           uint32_t *__restrict__ state)
{
    const uint32_t t = threadIdx.x;
    const uint32_t T = blockDim.x;
    const uint32_t span = T * SPL;   // slots written per round
    uint32_t base = 0;
    uint64_t i0 = 0;
    while (i0 < n) {
        const uint64_t left = n - i0;
        const uint32_t cnt = left < W ? (uint32_t)left : W;
        if (base + N + span > L) {
            // base > L - N - span >= N: source and destination are disjoint
            for (uint32_t k = t; k < N; k += T)
                X[k] = X[base + k];
            __syncthreads();
            base = 0;
        }
        round_steps<KIND, SPL>(X + base, rec, otb, N, M, sh1, sh2, mask, t, T, cnt, out + i0);
        __syncthreads();
        base += cnt;
        i0 += cnt;
    }
    // x_n .. x_{n+N-1} back to HBM (section 8: the next call continues)
    for (uint32_t k = t; k < N; k += T)
        state[k] = X[base + k];
}

template <int SPL>
__global__ __launch_bounds__(1024) void mtgp_generate_kernel(const GenRecord *__restrict__ recs,
                                                             uint32_t *__restrict__ states,
                                                             const WorkItem *__restrict__ items,
                                                             uint32_t nitems, uint32_t *counters,
                                                             WorkItem single, uint32_t L)
{
    extern __shared__ uint32_t smem[];
    uint32_t *rec = smem;
    uint32_t *otb = smem + 16;
    uint32_t *slot = smem + 32;
    uint32_t *X = smem + kTableWords;
    const uint32_t t = threadIdx.x;
    const uint32_t T = blockDim.x;

    for (uint32_t iter = 0;; ++iter) {
        WorkItem it;
        if (items == nullptr) {                 // one item passed by value, grid of 1
            if (iter > 0)
                break;
            it = single;
        } else if (counters == nullptr) {       // item i in workgroup i
            if (iter > 0 || blockIdx.x >= nitems)
                break;
            it = items[blockIdx.x];
        } else {                                // persistent: pop from the queue
            if (t == 0)
                slot[0] = atomicAdd(&counters[0], 1u);
            __syncthreads();
            const uint32_t q = __builtin_amdgcn_readfirstlane(slot[0]);
            __syncthreads();
            if (q >= nitems)
                break;
            it = items[q];
        }
        const uint32_t gen = __builtin_amdgcn_readfirstlane(it.gen);
        const uint32_t kind = __builtin_amdgcn_readfirstlane(it.kind);
        const GenRecord &g = recs[gen];
        const uint32_t N = g.N, M = g.M;
        uint32_t *state = states + g.state_off;
        const uint32_t W = (N - M) < T * SPL ? (N - M) : T * SPL;

        for (uint32_t k = t; k < N; k += T)
            X[k] = state[k];
        if (t < 16) {
            rec[t] = g.rec[t];
            otb[t] = kind == 0 ? g.tmp[t] : g.flt[t];
        }
        __syncthreads();

        gu32 *out = reinterpret_cast<gu32 *>(it.out);
        if (kind == 0)
            run_stream<0, SPL>(X, rec, otb, N, M, g.sh1, g.sh2, g.mask, W, L, it.n, out, state);
        else if (kind == 1)
            run_stream<1, SPL>(X, rec, otb, N, M, g.sh1, g.sh2, g.mask, W, L, it.n, out, state);
        else
            run_stream<2, SPL>(X, rec, otb, N, M, g.sh1, g.sh2, g.mask, W, L, it.n, out, state);
        __syncthreads();   // the next item overwrites the window and tables
    }

    if (items != nullptr && counters != nullptr && t == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&counters[1], 1u);
        if (done == gridDim.x - 1) {    // every pop has returned: reset for the next launch
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
}

// ---------------------------------------------------------------------------
// Wave form: each wavefront of the workgroup serves its own generator. The
// 64 lanes take steps k = lane + 64c (c < SPL) of each round. LDS operations
// of one wavefront complete in issue order, so a round's reads see the
// previous round's writes without a barrier or an LDS wait; the SPL
// independent steps per lane hide the LDS latency instead.
// LDS per wavefront: [0,16) recursion table, [16,32) output table, then the
// window X of L words.
// ---------------------------------------------------------------------------

template <int KIND, int SPL>
__device__ __forceinline__ void run_stream_wave(uint32_t *__restrict__ X, const uint32_t *__restrict__ rec,
                                                const uint32_t *__restrict__ otb, uint32_t N, uint32_t M,
                                                uint32_t sh1, uint32_t sh2, uint32_t mask, uint32_t W,
                                                uint32_t L, uint64_t n, gu32 *__restrict__ out,
                                                uint32_t *__restrict__ state, uint32_t lane)
{
    constexpr uint32_t span = 64u * SPL;
    uint32_t base = 0;
    uint64_t i0 = 0;
    while (i0 < n) {
        const uint64_t left = n - i0;
        const uint32_t cnt = left < W ? (uint32_t)left : W;
        if (base + N + span > L) {
            for (uint32_t k = lane; k < N; k += 64)
                X[k] = X[base + k];
            base = 0;
        }
        round_steps<KIND, SPL>(X + base, rec, otb, N, M, sh1, sh2, mask, lane, 64u, cnt, out + i0);
        base += cnt;
        i0 += cnt;
    }
    for (uint32_t k = lane; k < N; k += 64)
        state[k] = X[base + k];
}

template <int SPL>
__global__ __launch_bounds__(1024) void mtgp_wave_kernel(const GenRecord *__restrict__ recs,
                                                         uint32_t *__restrict__ states,
                                                         const WorkItem *__restrict__ items,
                                                         uint32_t nitems, uint32_t *counters,
                                                         WorkItem single, uint32_t L)
{
    extern __shared__ uint32_t smem[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t waves = blockDim.x >> 6;
    uint32_t *rec = smem + wave * (kTableWords + L);
    uint32_t *otb = rec + 16;
    uint32_t *X = rec + kTableWords;

    for (uint32_t iter = 0;; ++iter) {
        WorkItem it;
        if (items == nullptr) {                 // one item passed by value, one wavefront
            if (iter > 0 || blockIdx.x > 0 || wave > 0)
                break;
            it = single;
        } else if (counters == nullptr) {       // item i in wavefront i
            const uint32_t w = blockIdx.x * waves + wave;
            if (iter > 0 || w >= nitems)
                break;
            it = items[w];
        } else {                                // persistent: each wavefront pops its own item
            uint32_t q = 0;
            if (lane == 0)
                q = atomicAdd(&counters[0], 1u);
            q = __builtin_amdgcn_readfirstlane(q);
            if (q >= nitems)
                break;
            it = items[q];
        }
        const uint32_t gen = __builtin_amdgcn_readfirstlane(it.gen);
        const uint32_t kind = __builtin_amdgcn_readfirstlane(it.kind);
        const GenRecord &g = recs[gen];
        const uint32_t N = g.N, M = g.M;
        uint32_t *state = states + g.state_off;
        const uint32_t W = (N - M) < 64u * SPL ? (N - M) : 64u * SPL;

        for (uint32_t k = lane; k < N; k += 64)
            X[k] = state[k];
        if (lane < 16) {
            rec[lane] = g.rec[lane];
            otb[lane] = kind == 0 ? g.tmp[lane] : g.flt[lane];
        }
        gu32 *out = reinterpret_cast<gu32 *>(it.out);
        if (kind == 0)
            run_stream_wave<0, SPL>(X, rec, otb, N, M, g.sh1, g.sh2, g.mask, W, L, it.n, out, state, lane);
        else if (kind == 1)
            run_stream_wave<1, SPL>(X, rec, otb, N, M, g.sh1, g.sh2, g.mask, W, L, it.n, out, state, lane);
        else
            run_stream_wave<2, SPL>(X, rec, otb, N, M, g.sh1, g.sh2, g.mask, W, L, it.n, out, state, lane);
    }

    if (items != nullptr && counters != nullptr && lane == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&counters[1], 1u);
        if (done == gridDim.x * waves - 1) {    // every pop has returned: reset for the next launch
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
    if (shape.mode == kModeGroup) {
        const size_t lds = (size_t)(kTableWords + L) * sizeof(uint32_t);
#define MTGP_LAUNCH_GROUP(S)                                                                          \
    hipLaunchKernelGGL(mtgp_generate_kernel<S>, grid, block, lds, stream, recs, states, items, nitems, \
                       counters, single, L)
        switch (shape.spl) {
        case 1: MTGP_LAUNCH_GROUP(1); break;
        case 2: MTGP_LAUNCH_GROUP(2); break;
        case 4: MTGP_LAUNCH_GROUP(4); break;
        default: return hipErrorInvalidValue;
        }
#undef MTGP_LAUNCH_GROUP
    } else {
        const size_t lds = (size_t)(shape.threads / 64) * (kTableWords + L) * sizeof(uint32_t);
#define MTGP_LAUNCH_WAVE(S)                                                                           \
    hipLaunchKernelGGL(mtgp_wave_kernel<S>, grid, block, lds, stream, recs, states, items, nitems,     \
                       counters, single, L)
        switch (shape.spl) {
        case 1: MTGP_LAUNCH_WAVE(1); break;
        case 2: MTGP_LAUNCH_WAVE(2); break;
        case 4: MTGP_LAUNCH_WAVE(4); break;
        case 6: MTGP_LAUNCH_WAVE(6); break;
        case 8: MTGP_LAUNCH_WAVE(8); break;
        case 12: MTGP_LAUNCH_WAVE(12); break;
        case 16: MTGP_LAUNCH_WAVE(16); break;
        default: return hipErrorInvalidValue;
        }
#undef MTGP_LAUNCH_WAVE
    }
    return hipGetLastError();
}

hipError_t opt_in_lds(size_t bytes)
{
    const int b = (int)bytes;
    hipError_t e = hipSuccess;
#define MTGP_OPT_IN(K)                                                                            \
    if (e == hipSuccess)                                                                          \
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&K), hipFuncAttributeMaxDynamicSharedMemorySize, b)
    MTGP_OPT_IN(mtgp_generate_kernel<1>);
    MTGP_OPT_IN(mtgp_generate_kernel<2>);
    MTGP_OPT_IN(mtgp_generate_kernel<4>);
    MTGP_OPT_IN(mtgp_wave_kernel<1>);
    MTGP_OPT_IN(mtgp_wave_kernel<2>);
    MTGP_OPT_IN(mtgp_wave_kernel<4>);
    MTGP_OPT_IN(mtgp_wave_kernel<6>);
    MTGP_OPT_IN(mtgp_wave_kernel<8>);
    MTGP_OPT_IN(mtgp_wave_kernel<12>);
    MTGP_OPT_IN(mtgp_wave_kernel<16>);
#undef MTGP_OPT_IN
    return e;
}

}  // namespace mtgp_impl
