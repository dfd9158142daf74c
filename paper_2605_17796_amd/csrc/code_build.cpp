// Host construction of the quantum Tanner code and of the kernel tables.
//
//  * Left-right Cayley complex (Sec. II-A): a face for every (g, a, b),
//    {(g,0), (ag,1), (gb,1), (agb,0)}; TNC (ag != gb) makes the four corners
//    distinct and the faces at each vertex correspond to A x B.
//  * Z generators C_A (x) C_B on every V0 view, X generators
//    C_A^perp (x) C_B^perp on every V1 view (Sec. II-B).
//
// A face has exactly two V0 descriptions: (g, i, j) and
// (A_i g B_j, i*, j*) with A_{i*} = A_i^-1, B_{j*} = B_j^-1.  The qubit id of
// a face is the rank of its lexicographically smaller description.  The V1
// view of h lists, at local position (i, j), the face whose (g B_j', 1)
// corner is (h, 1), i.e. the description (h B_j, i, j*).
#include "code_build.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace lead {
namespace {

enum { kOk = 0, kArg = -1, kGroup = -2, kSym = -3, kTnc = -4, kLocal = -5 };

int popc(uint64_t x) { return __builtin_popcountll(x); }

// Row-reduce `rows` (each < 2^width) in place to reduced echelon form with
// pivots in increasing column order; returns the rank.
int rref_small(std::vector<uint64_t> &rows, int width) {
    int rank = 0;
    for (int col = 0; col < width && rank < (int)rows.size(); ++col) {
        const uint64_t bit = uint64_t(1) << col;
        int p = -1;
        for (int i = rank; i < (int)rows.size(); ++i)
            if (rows[i] & bit) { p = i; break; }
        if (p < 0) continue;
        std::swap(rows[p], rows[rank]);
        for (int i = 0; i < (int)rows.size(); ++i)
            if (i != rank && (rows[i] & bit)) rows[i] ^= rows[rank];
        ++rank;
    }
    rows.resize(rank);
    return rank;
}

// Basis (RREF) of {x : popcount(x & g) even for every row g}.
std::vector<uint64_t> dual_basis(const std::vector<uint64_t> &rref, int width) {
    std::vector<int> piv;
    for (uint64_t r : rref) piv.push_back(__builtin_ctzll(r));
    std::vector<uint64_t> out;
    for (int f = 0; f < width; ++f) {
        if (std::find(piv.begin(), piv.end(), f) != piv.end()) continue;
        uint64_t x = uint64_t(1) << f;
        for (size_t i = 0; i < rref.size(); ++i)
            if ((rref[i] >> f) & 1) x |= uint64_t(1) << piv[i];
        out.push_back(x);
    }
    rref_small(out, width);
    return out;
}

int min_weight(const std::vector<uint64_t> &basis) {
    int best = 1 << 30;
    const uint32_t n = 1u << basis.size();
    for (uint32_t s = 1; s < n; ++s) {
        uint64_t w = 0;
        for (size_t i = 0; i < basis.size(); ++i)
            if ((s >> i) & 1) w ^= basis[i];
        best = std::min(best, popc(w));
    }
    return best;
}

// GF(2) rank of a matrix with packed rows of `words` 64-bit words.
int packed_rank(std::vector<uint64_t> m, int rows, int words) {
    int rank = 0;
    for (int col = 0; col < words * 64 && rank < rows; ++col) {
        const int w = col >> 6;
        const uint64_t bit = uint64_t(1) << (col & 63);
        int p = -1;
        for (int i = rank; i < rows; ++i)
            if (m[(size_t)i * words + w] & bit) { p = i; break; }
        if (p < 0) continue;
        if (p != rank)
            for (int x = 0; x < words; ++x) std::swap(m[(size_t)p * words + x], m[(size_t)rank * words + x]);
        const uint64_t *pr = &m[(size_t)rank * words];
        for (int i = rank + 1; i < rows; ++i) {
            uint64_t *ri = &m[(size_t)i * words];
            if (ri[w] & bit)
                for (int x = w; x < words; ++x) ri[x] ^= pr[x];
        }
        ++rank;
    }
    return rank;
}

// sigma[j] = j' when the other occurrence of the qubit at local position j
// sits at position j' in every view; empty otherwise.
void position_map(int order, int d2, TypeTables &tt) {
    tt.sigma.assign(d2, -1);
    for (int s = 0; s < order * d2; ++s) {
        const int j = s % d2, jp = tt.partner[s] % d2;
        if (tt.sigma[j] < 0) tt.sigma[j] = jp;
        if (tt.sigma[j] != jp) { tt.sigma.clear(); return; }
    }
}

// Ownership of every qubit (see TypeTables).  The qubits not decided by the
// position rule are edges of a view multigraph, oriented along Euler tours
// of each component after pairing odd-degree views with auxiliary edges; the
// tail of each real edge owns the qubit.
void balanced_ownership(int order, int d2, TypeTables &tt) {
    const int nslots = order * d2;
    tt.owned.assign(nslots, 0);
    std::vector<int> cnt(order, 0);
    // edge e = qubit, endpoints = its two slots
    std::vector<std::pair<int, int>> edges;            // (slot a, slot b), a < b
    for (int s = 0; s < nslots; ++s) {
        if (s > tt.partner[s]) continue;
        const int j = s % d2;
        if (!tt.sigma.empty() && tt.sigma[j] != j) {
            const int own = j < tt.sigma[j] ? s : tt.partner[s];
            tt.owned[own] = 1;
            cnt[own / d2]++;
        } else {
            edges.push_back({s, tt.partner[s]});
        }
    }
    const int real = (int)edges.size();
    std::vector<std::vector<int>> inc(order);
    auto add = [&](int e, int u, int w) { inc[u].push_back(e); if (w != u) inc[w].push_back(e); };
    std::vector<std::pair<int, int>> ends;             // vertex endpoints of every edge
    for (int e = 0; e < real; ++e) {
        ends.push_back({edges[e].first / d2, edges[e].second / d2});
        add(e, ends[e].first, ends[e].second);
    }
    std::vector<int> odd;
    for (int v = 0; v < order; ++v)
        if (inc[v].size() % 2) odd.push_back(v);
    for (size_t i = 0; i + 1 < odd.size(); i += 2) {
        int e = (int)ends.size();
        ends.push_back({odd[i], odd[i + 1]});
        add(e, odd[i], odd[i + 1]);
    }
    std::vector<char> used(ends.size(), 0);
    std::vector<size_t> ptr(order, 0);
    std::vector<int> tail(ends.size(), -1);
    // iterative Hierholzer; records the direction in which each edge is walked
    for (int start = 0; start < order; ++start) {
        std::vector<std::pair<int, int>> stack;   // (vertex, edge used to arrive)
        stack.push_back({start, -1});
        while (!stack.empty()) {
            int u = stack.back().first;
            while (ptr[u] < inc[u].size() && used[inc[u][ptr[u]]]) ++ptr[u];
            if (ptr[u] == inc[u].size()) {
                stack.pop_back();
                continue;
            }
            int e = inc[u][ptr[u]++];
            used[e] = 1;
            int w = ends[e].first == u ? ends[e].second : ends[e].first;
            tail[e] = u;
            stack.push_back({w, e});
        }
    }
    for (int e = 0; e < real; ++e) {
        int a = edges[e].first, b = edges[e].second;
        int own = (tail[e] == a / d2) ? a : b;
        tt.owned[own] = 1;
        cnt[own / d2]++;
    }
    tt.own_max = *std::max_element(cnt.begin(), cnt.end());
}

}  // namespace

int build_code(int order, const uint16_t *mul, int delta, const int32_t *A, const int32_t *B, int kA,
               const uint64_t *GA, int kB, const uint64_t *GB, Code &c, std::string &err) {
    if (order < 1 || order > 65535 || !mul || !A || !B || !GA || !GB) { err = "bad argument"; return kArg; }
    if (delta < 2 || delta > kMaxDelta) { err = "delta must be in 2..8"; return kArg; }
    if (kA < 1 || kA >= delta || kB < 1 || kB >= delta) { err = "local dimensions must be in 1..delta-1"; return kArg; }
    const int N = order, D = delta, D2 = D * D;
    const size_t NN = (size_t)N * N;
    for (size_t i = 0; i < NN; ++i)
        if (mul[i] >= N) { err = "multiplication table entry out of range"; return kGroup; }
    auto M = [&](int a, int b) { return (int)mul[(size_t)a * N + b]; };

    // identity, inverses, associativity
    int e = -1;
    for (int x = 0; x < N && e < 0; ++x) {
        bool ok = true;
        for (int g = 0; g < N && ok; ++g) ok = M(x, g) == g && M(g, x) == g;
        if (ok) e = x;
    }
    if (e < 0) { err = "table has no identity"; return kGroup; }
    std::vector<int> inv(N, -1);
    for (int g = 0; g < N; ++g) {
        for (int h = 0; h < N; ++h)
            if (M(g, h) == e && M(h, g) == e) { inv[g] = h; break; }
        if (inv[g] < 0) { err = "element without inverse"; return kGroup; }
    }
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            const int ab = M(a, b);
            for (int x = 0; x < N; ++x)
                if (M(ab, x) != M(a, M(b, x))) { err = "table is not associative"; return kGroup; }
        }

    // generating sets
    std::vector<int> iotaA(D), iotaB(D);
    for (int s = 0; s < 2; ++s) {
        const int32_t *S = s ? B : A;
        std::vector<int> &iota = s ? iotaB : iotaA;
        for (int i = 0; i < D; ++i) {
            if (S[i] < 0 || S[i] >= N) { err = "generator index out of range"; return kArg; }
            if (S[i] == e) { err = std::string("identity in ") + (s ? "B" : "A"); return kSym; }
            for (int j = 0; j < i; ++j)
                if (S[j] == S[i]) { err = std::string("repeated element in ") + (s ? "B" : "A"); return kSym; }
        }
        for (int i = 0; i < D; ++i) {
            iota[i] = -1;
            for (int j = 0; j < D; ++j)
                if (S[j] == inv[S[i]]) iota[i] = j;
            if (iota[i] < 0) {
                err = std::string(s ? "B" : "A") + " is not closed under inverses (element " +
                      std::to_string(S[i]) + ")";
                return kSym;
            }
        }
    }
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j)
            for (int g = 0; g < N; ++g)
                if (M(A[i], g) == M(g, B[j])) {
                    err = "TNC fails: a*g == g*b for a=" + std::to_string(A[i]) + " g=" + std::to_string(g) +
                          " b=" + std::to_string(B[j]);
                    return kTnc;
                }

    // local codes
    std::vector<uint64_t> ga(GA, GA + kA), gb(GB, GB + kB);
    const uint64_t full = (D == 64) ? ~uint64_t(0) : ((uint64_t(1) << D) - 1);
    for (auto &x : ga) if (x & ~full) { err = "C_A row wider than delta"; return kLocal; }
    for (auto &x : gb) if (x & ~full) { err = "C_B row wider than delta"; return kLocal; }
    if (rref_small(ga, D) != kA || rref_small(gb, D) != kB) { err = "local generator matrix not full rank"; return kLocal; }
    std::vector<uint64_t> ha = dual_basis(ga, D), hb = dual_basis(gb, D);
    if (min_weight(ga) < 2 || min_weight(gb) < 2 || min_weight(ha) < 2 || min_weight(hb) < 2) {
        err = "local code or its dual has minimum distance < 2";
        return kLocal;
    }

    c.order = N; c.delta = D; c.kA = kA; c.kB = kB;
    c.mul.assign(mul, mul + NN);
    c.A.assign(A, A + D);
    c.B.assign(B, B + D);
    std::copy(ga.begin(), ga.end(), c.rrefA);
    std::copy(gb.begin(), gb.end(), c.rrefB);
    std::copy(ha.begin(), ha.end(), c.dualA);
    std::copy(hb.begin(), hb.end(), c.dualB);

    // faces -> qubit ids
    auto desc = [&](int g, int i, int j) { return (g * D + i) * D + j; };
    std::vector<int32_t> qid((size_t)N * D2, -1);
    int n = 0;
    for (int g = 0; g < N; ++g)
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                const int other = desc(M(M(A[i], g), B[j]), iotaA[i], iotaB[j]);
                const int self = desc(g, i, j);
                if (other == self) { err = "face with coincident corners"; return kTnc; }
                if (self < other) qid[self] = n++;
            }
    for (int g = 0; g < N; ++g)
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                const int other = desc(M(M(A[i], g), B[j]), iotaA[i], iotaB[j]);
                const int self = desc(g, i, j);
                if (self > other) qid[self] = qid[other];
            }
    c.n = n;

    for (int t = 0; t < 2; ++t) {
        TypeTables &tt = c.t[t];
        const std::vector<uint64_t> &ra = t == 0 ? ga : ha;
        const std::vector<uint64_t> &rb = t == 0 ? gb : hb;
        tt.r = (int)(ra.size() * rb.size());
        tt.mask.assign(tt.r, 0);
        for (size_t x = 0; x < ra.size(); ++x)
            for (size_t y = 0; y < rb.size(); ++y) {
                uint64_t m = 0;
                for (int a = 0; a < D; ++a)
                    if ((ra[x] >> a) & 1) m |= rb[y] << (a * D);
                tt.mask[x * rb.size() + y] = m;
            }
        tt.eloc = 0;
        for (uint64_t m : tt.mask) tt.eloc += popc(m);
        tt.view.assign((size_t)N * D2, 0);
        for (int g = 0; g < N; ++g)
            for (int i = 0; i < D; ++i)
                for (int j = 0; j < D; ++j)
                    tt.view[(size_t)g * D2 + i * D + j] =
                        t == 0 ? qid[desc(g, i, j)] : qid[desc(M(g, B[j]), i, iotaB[j])];
        // the two occurrences of every qubit
        std::vector<int> slot_a(n, -1), slot_b(n, -1);
        for (int s = 0; s < N * D2; ++s) {
            const int q = tt.view[s];
            if (slot_a[q] < 0) slot_a[q] = s;
            else if (slot_b[q] < 0) slot_b[q] = s;
            else { err = "qubit in more than two views"; return kTnc; }
        }
        tt.partner.assign((size_t)N * D2, -1);
        for (int q = 0; q < n; ++q) {
            if (slot_b[q] < 0) { err = "qubit in fewer than two views"; return kTnc; }
            tt.partner[slot_a[q]] = slot_b[q];
            tt.partner[slot_b[q]] = slot_a[q];
        }
        position_map(N, D2, tt);
        balanced_ownership(N, D2, tt);
        // global CSR
        const int m = N * tt.r;
        tt.csr_ptr.assign(m + 1, 0);
        tt.csr_idx.clear();
        for (int g = 0; g < N; ++g)
            for (int rho = 0; rho < tt.r; ++rho) {
                std::vector<int> cols;
                for (int jj = 0; jj < D2; ++jj)
                    if ((tt.mask[rho] >> jj) & 1) cols.push_back(tt.view[(size_t)g * D2 + jj]);
                std::sort(cols.begin(), cols.end());
                tt.csr_idx.insert(tt.csr_idx.end(), cols.begin(), cols.end());
                tt.csr_ptr[g * tt.r + rho + 1] = (int)tt.csr_idx.size();
            }
    }

    // CSS condition and ranks
    const int words = (n + 63) / 64;
    std::vector<uint64_t> P[2];
    for (int t = 0; t < 2; ++t) {
        const int m = N * c.t[t].r;
        P[t].assign((size_t)m * words, 0);
        for (int row = 0; row < m; ++row)
            for (int x = c.t[t].csr_ptr[row]; x < c.t[t].csr_ptr[row + 1]; ++x) {
                const int q = c.t[t].csr_idx[x];
                P[t][(size_t)row * words + q / 64] |= uint64_t(1) << (q % 64);
            }
    }
    const int mz = N * c.t[0].r, mx = N * c.t[1].r;
    for (int x = 0; x < mx; ++x)
        for (int z = 0; z < mz; ++z) {
            int par = 0;
            for (int w = 0; w < words; ++w) par ^= popc(P[1][(size_t)x * words + w] & P[0][(size_t)z * words + w]);
            if (par & 1) { err = "CSS condition fails"; return kLocal; }
        }
    for (int t = 0; t < 2; ++t) c.t[t].rank = packed_rank(P[t], N * c.t[t].r, words);
    c.k = n - c.t[0].rank - c.t[1].rank;
    return kOk;
}

}  // namespace lead
