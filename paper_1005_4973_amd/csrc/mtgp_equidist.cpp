// Dimension of equidistribution k(v), v = 1..32, of an MTGP parameter set
// (section 3.4's definitions), on the host, by lattice reduction over F2[t].
//
// For a generator of full period 2^p - 1 the state transition F has an
// irreducible characteristic polynomial phi of degree p. Bit j (j = 0 the
// MSB) of output i is c_j F^i x for a linear functional c_j on the state x.
// The v MSBs of k consecutive outputs are k-dimensionally equidistributed
// exactly when the k v functionals c_j F^i (i < k, j < v) are linearly
// independent, i.e. when no nonzero polynomial vector (l_0 .. l_{v-1}) with
// every deg l_j < k satisfies sum_j c_j l_j(F) = 0.
//
// Fix one nonzero state and let G_j(t) = sum_i b_j(i) t^{-i-1} be the
// generating function of its bit-j sequence; G_j = h_j / phi with
// deg h_j < p. Since the orbit of any nonzero state spans the state space,
// sum_j c_j l_j(F) = 0 holds exactly when sum_j l_j h_j = 0 mod phi. These
// vectors l form a lattice L_v in F2[t]^v with basis
//     (phi, 0, .., 0) and (g_j, e_j), g_j = h_j h_0^{-1} mod phi (0 < j < v),
// and k(v) is the least max-degree of a nonzero vector of L_v. A basis in
// weak Popov form (Mulders and Storjohann, 2003) is row reduced, so that
// least degree is its smallest row degree. L_{v+1} is L_v (with a zero
// last coordinate) plus the row (g_v, e_v), so the reduction is carried
// from one v to the next. This is the dual of the lattice view the paper's
// SIS method works in; it gives the same k(v).
#include "../../include/mtgp.h"
#include "mtgp_f2.h"

#include <algorithm>
#include <new>
#include <vector>

namespace mtgp_impl {
namespace {

using f2::Poly;

bool linear_table(const uint32_t *tbl)
{
    if (tbl[0] != 0)
        return false;
    for (int a = 0; a < 16; a++)
        for (int b = 0; b < 16; b++)
            if (tbl[a ^ b] != (tbl[a] ^ tbl[b]))
                return false;
    return true;
}

bool prime(uint32_t v)
{
    if (v < 2)
        return false;
    for (uint32_t d = 2; d * d <= v; d++)
        if (v % d == 0)
            return false;
    return true;
}

// n outputs (tempered when `tempered`, else the raw words x_{i+N}) of the
// recursion from the state seeded with the library's seeding recurrence.
std::vector<uint32_t> host_outputs(const mtgp_param_set &ps, bool tempered, size_t n)
{
    const uint32_t N = (ps.mexp + 31) / 32;
    const uint32_t mask = 0xffffffffu << (32 * N - ps.mexp);
    std::vector<uint32_t> x((size_t)N + n);
    uint32_t v = 1u;
    x[0] = v;
    for (uint32_t i = 1; i < N; i++) {
        v = 1812433253u * (v ^ (v >> 30)) + i;
        x[i] = v;
    }
    std::vector<uint32_t> out(n);
    for (size_t i = 0; i < n; i++) {
        uint32_t t = x[i + 1] ^ (x[i] & mask);
        t ^= t << ps.sh1;
        const uint32_t u = t ^ (x[i + ps.pos] >> ps.sh2);
        const uint32_t y = u ^ ps.param_tbl[u & 0xf];
        x[i + N] = y;
        if (tempered) {
            uint32_t s = x[i + ps.pos - 1] ^ (x[i + ps.pos - 1] >> 16);
            s ^= s >> 8;
            out[i] = y ^ ps.temper_tbl[s & 0xf];
        } else {
            out[i] = y;
        }
    }
    return out;
}

Poly add(const Poly &a, const Poly &b)
{
    Poly r = a.w.size() >= b.w.size() ? a : b;
    const Poly &s = a.w.size() >= b.w.size() ? b : a;
    for (size_t i = 0; i < s.w.size(); i++)
        r.w[i] ^= s.w[i];
    r.trim();
    return r;
}

// a^{-1} mod m for m irreducible and a != 0 mod m (extended Euclid); the
// zero polynomial if a is not invertible.
Poly inverse_mod(const Poly &a, const Poly &m)
{
    Poly r0 = m, r1 = f2::mod(a, m);
    Poly s0, s1 = Poly::one();
    while (r1.deg > 0) {
        Poly r;
        const Poly q = f2::divide(r0, r1, &r);
        r0 = r1;
        r1 = r;
        Poly s = add(s0, f2::mul(q, s1));
        s0 = s1;
        s1 = s;
    }
    if (r1.deg != 0)
        return Poly();
    return f2::mod(s1, m);
}

// A lattice row: `cols` polynomial components of at most `W` words each.
struct Row {
    std::vector<uint64_t> c;
    std::vector<int32_t> deg;   // -1 for a zero component
};

class Lattice {
public:
    Lattice(uint32_t maxcols, int64_t maxdeg) : maxcols_(maxcols), W_((size_t)(maxdeg / 64 + 2)) {}

    // Add a row given by its components (at most cols() + 1 of them; a new
    // column is opened when it has cols() + 1) and restore weak Popov form.
    // Returns false if a row became zero (the rows were dependent).
    bool insert(const std::vector<Poly> &comps)
    {
        cols_ = std::max<uint32_t>(cols_, (uint32_t)comps.size());
        Row r;
        r.c.assign((size_t)maxcols_ * W_, 0);
        r.deg.assign(maxcols_, -1);
        for (size_t j = 0; j < comps.size(); j++) {
            for (size_t k = 0; k < comps[j].w.size() && k < W_; k++)
                r.c[j * W_ + k] = comps[j].w[k];
            r.deg[j] = (int32_t)comps[j].deg;
        }
        rows_.push_back(std::move(r));
        owner_.resize(maxcols_, -1);
        std::vector<size_t> todo{rows_.size() - 1};
        while (!todo.empty()) {
            size_t a = todo.back();
            todo.pop_back();
            for (;;) {
                const int32_t da = row_deg(a);
                if (da < 0)
                    return false;
                const uint32_t l = pivot(a, da);
                const int64_t b = owner_[l];
                if (b < 0) {
                    owner_[l] = (int64_t)a;
                    break;
                }
                const int32_t db = row_deg((size_t)b);
                if (da >= db) {
                    add_shifted(a, (size_t)b, da - db);
                } else {
                    add_shifted((size_t)b, a, db - da);
                    owner_[l] = (int64_t)a;
                    todo.push_back((size_t)b);
                    break;
                }
            }
        }
        return true;
    }

    // Least row degree: the least max-degree of a nonzero lattice vector.
    int32_t shortest() const
    {
        int32_t best = -1;
        for (size_t i = 0; i < rows_.size(); i++) {
            const int32_t d = row_deg(i);
            if (best < 0 || d < best)
                best = d;
        }
        return best;
    }

private:
    int32_t row_deg(size_t i) const
    {
        int32_t d = -1;
        for (uint32_t j = 0; j < cols_; j++)
            d = std::max(d, rows_[i].deg[j]);
        return d;
    }
    // the last column holding the row degree
    uint32_t pivot(size_t i, int32_t d) const
    {
        uint32_t l = 0;
        for (uint32_t j = 0; j < cols_; j++)
            if (rows_[i].deg[j] == d)
                l = j;
        return l;
    }
    // row a += t^s row b (s >= 0, row degrees then equal at most deg a)
    void add_shifted(size_t a, size_t b, int32_t s)
    {
        Row &ra = rows_[a];
        const Row &rb = rows_[b];
        const size_t ws = (size_t)s >> 6;
        const int bs = s & 63;
        for (uint32_t j = 0; j < cols_; j++) {
            if (rb.deg[j] < 0)
                continue;
            uint64_t *dst = ra.c.data() + (size_t)j * W_;
            const uint64_t *src = rb.c.data() + (size_t)j * W_;
            const size_t n = (size_t)rb.deg[j] / 64 + 1;
            if (bs == 0) {
                for (size_t k = 0; k < n; k++)
                    dst[ws + k] ^= src[k];
            } else {
                uint64_t carry = 0;
                for (size_t k = 0; k < n; k++) {
                    dst[ws + k] ^= (src[k] << bs) | carry;
                    carry = src[k] >> (64 - bs);
                }
                if (carry)
                    dst[ws + n] ^= carry;
            }
            int32_t top = std::max(ra.deg[j], rb.deg[j] + s);
            int64_t w = top / 64;
            int32_t d = -1;
            for (; w >= 0; w--)
                if (dst[w]) {
                    d = (int32_t)(w * 64 + 63 - __builtin_clzll(dst[w]));
                    break;
                }
            ra.deg[j] = d;
        }
    }

    uint32_t maxcols_;
    size_t W_;
    uint32_t cols_ = 0;
    std::vector<Row> rows_;
    std::vector<int64_t> owner_;
};

}  // namespace
}  // namespace mtgp_impl

using namespace mtgp_impl;

extern "C" int mtgp_equidistribution(const mtgp_param_set *ps, uint32_t tempered, uint32_t vmax, uint32_t *k,
                                     uint32_t *delta)
{
    if (!ps || !k || vmax < 1 || vmax > 32 || !prime(ps->mexp) || ps->mexp < 67 || ps->mexp > 65536)
        return MTGP_EINVAL;
    const uint32_t p = ps->mexp;
    const uint32_t N = (p + 31) / 32;
    if (ps->pos < 2 || ps->pos > N - 1 || ps->sh1 > 31 || ps->sh2 > 31 || !linear_table(ps->param_tbl) ||
        !linear_table(ps->temper_tbl))
        return MTGP_EINVAL;
    try {
        // characteristic polynomial: minimal polynomial of the MSB sequence,
        // which is phi itself when phi is irreducible of degree p
        const size_t nbits = 2 * (size_t)p + 64;
        const std::vector<uint32_t> out = host_outputs(*ps, tempered != 0, nbits);
        std::vector<uint64_t> msb(nbits / 64 + 1, 0);
        for (size_t i = 0; i < nbits; i++)
            if (out[i] >> 31)
                msb[i >> 6] |= 1ull << (i & 63);
        const Poly phi = f2::minpoly(msb.data(), (int64_t)nbits);
        bool sieved = false;
        if (phi.deg != (int64_t)p || !f2::irreducible_prime_degree(phi, 28, &sieved))
            return MTGP_EINVAL;   // period is not 2^p - 1: k(v) is not defined as in section 3.4

        // h_j = (phi * B_j) >> p with B_j the first p bits of plane j reversed
        std::vector<Poly> h(vmax);
        for (uint32_t j = 0; j < vmax; j++) {
            std::vector<uint64_t> rev(p / 64 + 1, 0);
            for (uint32_t i = 0; i < p; i++)
                if ((out[i] >> (31 - j)) & 1)
                    rev[(p - 1 - i) >> 6] |= 1ull << ((p - 1 - i) & 63);
            const Poly prod = f2::mul(phi, Poly::from_words(rev.data(), (int64_t)p - 1));
            Poly hj;
            if (prod.deg >= (int64_t)p) {
                hj.w.assign((size_t)((prod.deg - p) / 64 + 1), 0);
                for (int64_t m = 0; m <= prod.deg - (int64_t)p; m++)
                    if (prod.bit(m + p))
                        hj.w[(size_t)(m >> 6)] |= 1ull << (m & 63);
                hj.trim();
            }
            h[j] = hj;
        }
        if (h[0].deg < 0) {
            // the MSB sequence vanishes: not even 1-dimensionally equidistributed
            for (uint32_t v = 1; v <= vmax; v++)
                k[v - 1] = 0;
        } else {
            const Poly inv = inverse_mod(h[0], phi);
            if (inv.deg < 0)
                return MTGP_EINVAL;
            Lattice lat(vmax, (int64_t)p);
            if (!lat.insert({phi}))
                return MTGP_EINVAL;
            k[0] = (uint32_t)lat.shortest();
            for (uint32_t v = 2; v <= vmax; v++) {
                std::vector<Poly> row(v);
                row[0] = f2::mulmod(h[v - 1], inv, phi);
                row[v - 1] = Poly::one();
                if (!lat.insert(row))
                    return MTGP_EINVAL;
                k[v - 1] = (uint32_t)lat.shortest();
            }
        }
        if (delta) {
            uint32_t d = 0;
            for (uint32_t v = 1; v <= vmax; v++)
                d += p / v - std::min(p / v, k[v - 1]);
            *delta = d;
        }
        return MTGP_OK;
    } catch (const std::bad_alloc &) {
        return MTGP_ENOMEM;
    }
}
