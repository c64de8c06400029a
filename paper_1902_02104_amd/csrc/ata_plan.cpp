// Host planner: turns the ATA recursion (Section 3, Algorithm 1) into a
// device task table.
//
// The recursion splits the rows of every sub-problem as well as its columns.
// A row split only produces a sum (C11 = A11^t A11 + A21^t A21, the "second
// product accumulated into the first"), so row chunks that share the same
// column structure become one task whose K loop runs over their row segments
// in order.  Every scalar product of the paper's recursion tree is formed; only
// the order in which products of different row chunks are summed changes.
// Chunks whose sub-trees differ (a row count straddling the cutoff) are kept
// in separate groups that write the same output in successive phases.
//
// HASA (the rectangular Strassen routine for the off-diagonal block) splits
// M, K and N into ceil/floor halves with implicit zero padding.  The top
// (d - 1) of its d levels are expanded here into signed operand terms that
// the kernels sum while staging tiles; the last level is done inside each
// workgroup tile; products of expanded levels go to a workspace and a
// combination kernel forms the result quadrants.
#include "ata_plan.h"

#include <algorithm>
#include <map>
#include <stdexcept>

namespace atalib {

// Strassen 1969 (variant 0): M1 = (L11 + L22)(R11 + R22), M2 = (L21 + L22) R11,
// M3 = L11 (R12 - R22), M4 = L22 (R21 - R11), M5 = (L11 + L12) R22,
// M6 = (L21 - L11)(R11 + R12), M7 = (L12 - L22)(R21 + R22);
// D11 = M1 + M4 - M5 + M7, D12 = M3 + M5, D21 = M2 + M4, D22 = M1 - M2 + M3 + M6.
// Winograd 1971 (variant 1): P1 = L11 R11, P2 = L12 R21, P3 = S4 R22,
// P4 = L22 T4, P5 = S1 T1, P6 = S2 T2, P7 = S3 T3 with S1 = L21 + L22,
// S2 = S1 - L11, S3 = L11 - L21, S4 = L12 - S2, T1 = R12 - R11, T2 = R22 - T1,
// T3 = R22 - R12, T4 = T2 - R21; D11 = P1 + P2, D12 = P1 + P6 + P5 + P3,
// D21 = P1 + P6 + P7 - P4, D22 = P1 + P6 + P7 + P5.
// Index order: x_coef [a*2+b] for L_ab, y_coef [b*2+c] for R_bc, d_coef [a*2+c].
const int x_coef[2][7][4] = {
    {{1, 0, 0, 1}, {0, 0, 1, 1}, {1, 0, 0, 0}, {0, 0, 0, 1}, {1, 1, 0, 0}, {-1, 0, 1, 0}, {0, 1, 0, -1}},
    {{1, 0, 0, 0}, {0, 1, 0, 0}, {1, 1, -1, -1}, {0, 0, 0, 1}, {0, 0, 1, 1}, {-1, 0, 1, 1}, {1, 0, -1, 0}},
};
const int y_coef[2][7][4] = {
    {{1, 0, 0, 1}, {1, 0, 0, 0}, {0, 1, 0, -1}, {-1, 0, 1, 0}, {0, 0, 0, 1}, {1, 1, 0, 0}, {0, 0, 1, 1}},
    {{1, 0, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}, {1, -1, -1, 1}, {-1, 1, 0, 0}, {1, -1, 0, 1}, {0, -1, 0, 1}},
};
const int d_coef[2][7][4] = ATA_D_COEF;

namespace {

inline int64_t ceil2(int64_t x) { return (x + 1) / 2; }
inline int64_t tri(int64_t x) { return x * (x + 1) / 2; }

struct Chunk {
    int64_t row, h;
};

// A term of an operand during symbolic expansion: a column range plus one row
// range per chunk.
struct XTerm {
    int32_t sign;
    int64_t col, cvend;
    std::vector<int64_t> row, rvend;
};

struct Product {
    std::vector<XTerm> x, y;
};

class Builder {
public:
    Builder(Plan& p) : P(p), o(p.opt) {}

    int ata_node(const std::vector<Chunk>& chunks, int64_t c0, int64_t w, int phase, int level);

private:
    Plan& P;
    const PlanOptions& o;

    Phase& ph(int idx) {
        while ((int)P.phases.size() <= idx) P.phases.emplace_back();
        return P.phases[idx];
    }
    int hasa_block(const std::vector<Chunk>& chunks, int64_t xc, int64_t M, int64_t yc, int64_t N,
                   int phase);
    // Cost of a product in 128 x 128 x 1 tile steps at the measured rates:
    // classical tiles, or one Strassen level (seven half-size products in
    // product tiles of 128, or in-tile quadrants of 64, plus the combination).
    bool level_pays(int64_t M, int64_t K, int64_t N) const {
        auto t128 = [](int64_t x) { return (double)((x + kGemmTile - 1) / kGemmTile); };
        auto t64 = [](int64_t x) { return (double)((x + kStrTile - 1) / kStrTile); };
        const double classical = t128(M) * t128(N) * (double)K / o.rate_one;
        const int64_t MH = ceil2(M), NH = ceil2(N), KH = ceil2(K);
        const double prods = o.intile ? 7.0 / 4.0 * t64(MH) * t64(NH) * (double)KH
                                      : 7.0 * t128(MH) * t128(NH) * (double)KH;
        const double strassen = prods / o.rate_two + o.comb * (double)M * (double)N + o.eq * (double)(M + N) * (double)K;
        return strassen < classical;
    }
    int hasa_depth(int64_t M, int64_t K, int64_t N) const {
        int d = 0;
        while (std::min(M, std::min(K, N)) > o.cutoff && (o.max_depth < 0 || d < o.max_depth)) {
            if (o.adaptive && !level_pays(M, K, N)) break;
            M = ceil2(M);
            K = ceil2(K);
            N = ceil2(N);
            ++d;
        }
        return d;
    }
    void add_segments_merged(DevTask& t, const std::vector<Chunk>& chs);
    bool subtree_strassen(const std::vector<int64_t>& hs, int64_t w);
    std::map<std::vector<int64_t>, bool> strassen_memo;
    int32_t push_terms(const std::vector<XTerm>& x, const std::vector<XTerm>& y);
};

static void check32(int64_t v) {
    if (v < 0 || v > INT32_MAX) throw std::invalid_argument("dimension exceeds 32-bit range");
}

// Contiguous chunks form one segment: [row, row + klen) for both operands.
void Builder::add_segments_merged(DevTask& t, const std::vector<Chunk>& chs) {
    t.seg_off = (int32_t)P.segs.size();
    t.nseg = 0;
    size_t i = 0;
    while (i < chs.size()) {
        int64_t r = chs[i].row, e = chs[i].row + chs[i].h;
        size_t j = i + 1;
        while (j < chs.size() && chs[j].row == e) {
            e += chs[j].h;
            ++j;
        }
        check32(e);
        P.segs.push_back((int32_t)(e - r));  // klen
        P.segs.push_back(0);                 // window [0, klen)
        P.segs.push_back((int32_t)(e - r));
        P.segs.push_back((int32_t)r);
        P.segs.push_back((int32_t)e);
        P.segs.push_back((int32_t)r);
        P.segs.push_back((int32_t)e);
        ++t.nseg;
        i = j;
    }
}

int32_t Builder::push_terms(const std::vector<XTerm>& x, const std::vector<XTerm>& y) {
    int32_t off = (int32_t)P.terms.size();
    for (const auto* list : {&x, &y})
        for (const XTerm& t : *list) {
            check32(t.cvend);
            P.terms.push_back(DevTerm{(int32_t)t.col, (int32_t)t.cvend, t.sign, 0});
        }
    return off;
}

// Whether the subtree of a node of width w over row chunks of these heights
// takes a Strassen level anywhere (memoised on the width and the distinct
// heights).
bool Builder::subtree_strassen(const std::vector<int64_t>& hs, int64_t w) {
    std::vector<int64_t> key(hs);
    std::sort(key.begin(), key.end());
    key.erase(std::unique(key.begin(), key.end()), key.end());
    key.push_back(w);
    auto it = strassen_memo.find(key);
    if (it != strassen_memo.end()) return it->second;
    bool any = false;
    std::vector<int64_t> sub;
    for (size_t i = 0; i + 1 < key.size(); ++i) {
        const int64_t h = key[i];
        if (h <= o.cutoff || w <= o.cutoff) continue;
        sub.push_back(ceil2(h));
        if (h / 2 > 0) sub.push_back(h / 2);
    }
    if (!sub.empty()) {
        const int64_t n1 = ceil2(w), n2 = w / 2;
        for (int64_t h : sub) any = any || hasa_depth(n2, h, n1) > 0;
        any = any || subtree_strassen(sub, n1) || subtree_strassen(sub, n2);
    }
    strassen_memo[key] = any;
    return any;
}

int Builder::ata_node(const std::vector<Chunk>& chunks, int64_t c0, int64_t w, int phase,
                      int level) {
    std::vector<Chunk> leaf, rec;
    // A subtree without any Strassen level is a plain partition of the
    // classical product of its columns over its rows: it runs as one
    // diagonal block of the whole width (the same multiplications, in
    // larger tiles).
    bool flat = false;
    {
        std::vector<int64_t> hs;
        for (const Chunk& ch : chunks) hs.push_back(ch.h);
        flat = !subtree_strassen(hs, w);
    }
    for (const Chunk& ch : chunks) {
        if (flat || ch.h <= o.cutoff || w <= o.cutoff)
            leaf.push_back(ch);
        else
            rec.push_back(ch);
    }
    int next = phase;
    if (!rec.empty()) {
        if (level + 1 > P.ata_depth) P.ata_depth = level + 1;
        std::vector<Chunk> sub;
        sub.reserve(rec.size() * 2);
        for (const Chunk& ch : rec) {
            const int64_t h1 = ceil2(ch.h);
            sub.push_back(Chunk{ch.row, h1});          // rows of A11 / A12
            sub.push_back(Chunk{ch.row + h1, ch.h / 2});  // rows of A21 / A22
        }
        const int64_t n1 = ceil2(w), n2 = w / 2;
        int p1 = ata_node(sub, c0, n1, phase, level + 1);       // C11 = S1 + S2
        int p2 = ata_node(sub, c0 + n1, n2, phase, level + 1);  // C22 = S3 + S4
        int p3 = hasa_block(sub, c0 + n1, n2, c0, n1, phase);   // C21 = S5 + S6
        next = std::max(p1, std::max(p2, p3));
    }
    if (!leaf.empty()) {
        const int lp = rec.empty() ? phase : next;
        DevTask t{};
        t.kind = TK_SYRK;
        t.M = t.N = (int32_t)w;
        t.nx = t.ny = 1;
        t.term_off = push_terms({XTerm{1, c0, c0 + w, {}, {}}}, {XTerm{1, c0, c0 + w, {}, {}}});
        add_segments_merged(t, leaf);
        t.dst = 0;
        t.beta = rec.empty() ? 0 : 1;
        t.dM = t.dN = (int32_t)w;
        t.r0 = t.q0 = (int32_t)c0;
        const int64_t T = (w + kGemmTile - 1) / kGemmTile;
        t.tiles_m = t.tiles_n = (int32_t)T;
        int64_t ktot = 0;
        for (const Chunk& ch : leaf) ktot += ch.h;
        P.mults += tri(w) * ktot;
        P.syrk_mults += tri(w) * ktot;
        const int32_t id = (int32_t)P.tasks.size();
        P.tasks.push_back(t);
        for (int64_t ti = 0; ti < T; ++ti)
            for (int64_t tj = 0; tj <= ti; ++tj) ph(lp).syrk_items.push_back(WorkItem{id, (int32_t)ti, (int32_t)tj, 0});
        ++P.syrk_tasks;
        next = lp + 1;
    }
    return next;
}

int Builder::hasa_block(const std::vector<Chunk>& chunks, int64_t xc, int64_t M, int64_t yc,
                        int64_t N, int phase) {
    // group chunks by the HASA depth their shape gives (heaviest first)
    std::map<int, std::vector<Chunk>, std::greater<int>> groups;
    for (const Chunk& ch : chunks) groups[hasa_depth(M, ch.h, N)].push_back(ch);
    int gi = 0;
    for (auto& kv : groups) {
        const int d = kv.first;
        const std::vector<Chunk>& chs = kv.second;
        const int gphase = phase + gi;
        const int beta = gi > 0 ? 1 : 0;
        ++gi;
        if (d > P.max_hasa_depth) P.max_hasa_depth = d;
        int64_t ktot = 0;
        for (const Chunk& ch : chs) ktot += ch.h;
        if (d == 0) {
            DevTask t{};
            t.kind = TK_GEMM;
            t.M = (int32_t)M;
            t.N = (int32_t)N;
            t.nx = t.ny = 1;
            t.term_off = push_terms({XTerm{1, xc, xc + M, {}, {}}}, {XTerm{1, yc, yc + N, {}, {}}});
            add_segments_merged(t, chs);
            t.dst = 0;
            t.beta = beta;
            t.dM = (int32_t)M;
            t.dN = (int32_t)N;
            t.r0 = (int32_t)xc;
            t.q0 = (int32_t)yc;
            t.tiles_m = (int32_t)((M + kGemmTile - 1) / kGemmTile);
            t.tiles_n = (int32_t)((N + kGemmTile - 1) / kGemmTile);
            P.mults += M * N * ktot;
            P.gemm_mults += M * N * ktot;
            const int32_t id = (int32_t)P.tasks.size();
            P.tasks.push_back(t);
            for (int32_t a = 0; a < t.tiles_m; ++a)
                for (int32_t b = 0; b < t.tiles_n; ++b) ph(gphase).gemm_items.push_back(WorkItem{id, a, b, 0});
            ++P.gemm_tasks;
            continue;
        }
        // symbolic expansion of the top d-1 levels (all d for product tiles)
        // (Winograd operands reach four terms per level: one level only)
        const bool tiled = !o.intile && d <= (o.variant == 0 ? kMaxExpandDepth : 1);
        const int expand = tiled ? d : d - 1;
        const size_t nch = chs.size();
        XTerm x0{1, xc, xc + M, {}, {}}, y0{1, yc, yc + N, {}, {}};
        std::vector<int64_t> K(nch);
        for (size_t c = 0; c < nch; ++c) {
            x0.row.push_back(chs[c].row);
            x0.rvend.push_back(chs[c].row + chs[c].h);
            K[c] = chs[c].h;
        }
        y0.row = x0.row;
        y0.rvend = x0.rvend;
        std::vector<Product> prods{Product{{x0}, {y0}}};
        int64_t Mp = M, Np = N;
        for (int lev = 1; lev <= expand; ++lev) {
            const int64_t MH = ceil2(Mp), NH = ceil2(Np);
            std::vector<int64_t> KH(nch);
            for (size_t c = 0; c < nch; ++c) KH[c] = ceil2(K[c]);
            std::vector<Product> next;
            next.reserve(prods.size() * 7);
            for (const Product& pr : prods) {
                for (int p = 0; p < 7; ++p) {
                    Product q;
                    for (int ab = 0; ab < 4; ++ab) {
                        const int cf = x_coef[o.variant][p][ab];
                        if (!cf) continue;
                        const int a = ab >> 1, b = ab & 1;
                        for (const XTerm& t : pr.x) {
                            XTerm u;
                            u.sign = t.sign * cf;
                            u.col = t.col + a * MH;
                            u.cvend = a == 0 ? std::min(t.cvend, t.col + MH) : t.cvend;
                            if (u.cvend <= u.col) continue;  // all-zero quadrant
                            bool any = false;
                            for (size_t c = 0; c < nch; ++c) {
                                const int64_t r = t.row[c] + b * KH[c];
                                const int64_t e = b == 0 ? std::min(t.rvend[c], t.row[c] + KH[c]) : t.rvend[c];
                                u.row.push_back(r);
                                u.rvend.push_back(std::max(r, e));
                                any |= e > r;
                            }
                            if (any) q.x.push_back(u);
                        }
                    }
                    for (int bc = 0; bc < 4; ++bc) {
                        const int cf = y_coef[o.variant][p][bc];
                        if (!cf) continue;
                        const int b = bc >> 1, cc = bc & 1;
                        for (const XTerm& t : pr.y) {
                            XTerm u;
                            u.sign = t.sign * cf;
                            u.col = t.col + cc * NH;
                            u.cvend = cc == 0 ? std::min(t.cvend, t.col + NH) : t.cvend;
                            if (u.cvend <= u.col) continue;
                            bool any = false;
                            for (size_t c = 0; c < nch; ++c) {
                                const int64_t r = t.row[c] + b * KH[c];
                                const int64_t e = b == 0 ? std::min(t.rvend[c], t.row[c] + KH[c]) : t.rvend[c];
                                u.row.push_back(r);
                                u.rvend.push_back(std::max(r, e));
                                any |= e > r;
                            }
                            if (any) q.y.push_back(u);
                        }
                    }
                    next.push_back(std::move(q));
                }
            }
            prods.swap(next);
            Mp = MH;
            Np = NH;
            K = KH;
        }
        const bool direct = !tiled && d == 1;
        const int64_t ws_base = P.ws_elems;
        if (!direct) P.ws_elems += (int64_t)prods.size() * Mp * Np;
        const int64_t MHin = ceil2(Mp), NHin = ceil2(Np);
        int64_t khalf = 0, kfull = 0;
        for (size_t c = 0; c < nch; ++c) {
            khalf += ceil2(K[c]);
            kfull += K[c];
        }
        const int32_t group = tiled ? P.n_groups++ : -1;
        for (size_t s = 0; tiled && s < prods.size(); ++s) {
            // product s of the fully expanded recursion as a classical tile task
            const Product& pr = prods[s];
            if ((int)pr.x.size() > kMaxTerms || (int)pr.y.size() > kMaxTerms)
                throw std::length_error("Strassen depth needs more operand terms than supported");
            DevTask t{};
            t.kind = TK_GEMM;
            t.variant = o.variant;
            t.M = (int32_t)Mp;
            t.N = (int32_t)Np;
            t.nx = (int32_t)pr.x.size();
            t.ny = (int32_t)pr.y.size();
            t.term_off = push_terms(pr.x, pr.y);
            t.seg_off = (int32_t)P.segs.size();
            t.nseg = (int32_t)nch;
            for (size_t c = 0; c < nch; ++c) {
                check32(K[c]);
                P.segs.push_back((int32_t)K[c]);  // klen
                P.segs.push_back(0);              // window [0, klen)
                P.segs.push_back((int32_t)K[c]);
                for (const auto* list : {&pr.x, &pr.y})
                    for (const XTerm& u : *list) {
                        check32(u.rvend[c]);
                        P.segs.push_back((int32_t)u.row[c]);
                        P.segs.push_back((int32_t)u.rvend[c]);
                    }
            }
            t.dst = 1;
            t.beta = 0;
            t.dM = (int32_t)Mp;
            t.dN = (int32_t)Np;
            t.ws_off = ws_base + (int64_t)s * Mp * Np;
            t.tiles_m = (int32_t)((Mp + kGemmTile - 1) / kGemmTile);
            t.tiles_n = (int32_t)((Np + kGemmTile - 1) / kGemmTile);
            P.mults += Mp * Np * kfull;
            P.str_mults += Mp * Np * kfull;
            if (o.opsums) {
                // t only describes the sums; the launched task is classical on them
                const int32_t dsc = (int32_t)P.tasks.size();
                P.tasks.push_back(t);
                check32(kfull);
                check32(Mp + Np);
                DevOpSum os{dsc, (int32_t)kfull, (int32_t)Mp, (int32_t)Np, P.opsum_elems, ph(gphase).opsum_rows};
                int64_t c0 = 0;  // first column of the product's operands in their buffer
                if (o.lp) {
                    // rows of the converted operand copy; 64 x 64 conversion tiles
                    os.out_off = P.lp_ops_rows;
                    c0 = P.lp_ops_rows;
                    check32(P.lp_ops_rows + Mp + Np);
                    P.lp_ops_rows += Mp + Np;
                    P.lp_ops_k = std::max(P.lp_ops_k, kfull);
                    ph(gphase).opsum_rows += ((kfull + 63) / 64) * ((Mp + Np + 63) / 64);
                } else {
                    P.opsum_elems += kfull * (Mp + Np);
                    ph(gphase).opsum_rows += kfull;
                }
                ph(gphase).opsums.push_back(os);
                DevTask g = t;
                g.nx = g.ny = 1;
                g.term_off = push_terms({XTerm{1, c0, c0 + Mp, {}, {}}}, {XTerm{1, c0 + Mp, c0 + Mp + Np, {}, {}}});
                g.seg_off = (int32_t)P.segs.size();
                g.nseg = 1;
                for (int32_t v : {(int32_t)kfull, 0, (int32_t)kfull, 0, (int32_t)kfull, 0, (int32_t)kfull})
                    P.segs.push_back(v);
                g.src = 1;
                g.src_off = os.out_off;
                t = g;
            }
            const int32_t id = (int32_t)P.tasks.size();
            P.tasks.push_back(t);
            P.task_group.resize(P.tasks.size(), -1);
            P.task_group[id] = group;
            for (int32_t a = 0; a < t.tiles_m; ++a)
                for (int32_t b = 0; b < t.tiles_n; ++b) ph(gphase).tg_items.push_back(WorkItem{id, a, b, 0});
            ph(gphase).tg_tmax = std::max(ph(gphase).tg_tmax, std::max(t.nx, t.ny));
            ++P.str_tasks;
        }
        for (size_t s = 0; !tiled && s < prods.size(); ++s) {
            const Product& pr = prods[s];
            if ((int)pr.x.size() > kMaxTerms || (int)pr.y.size() > kMaxTerms)
                throw std::length_error("Strassen depth needs more operand terms than supported");
            DevTask t{};
            t.kind = TK_STR;
            t.variant = o.variant;
            t.M = (int32_t)Mp;
            t.N = (int32_t)Np;
            t.nx = (int32_t)pr.x.size();
            t.ny = (int32_t)pr.y.size();
            t.term_off = push_terms(pr.x, pr.y);
            t.seg_off = (int32_t)P.segs.size();
            t.nseg = (int32_t)nch;
            for (size_t c = 0; c < nch; ++c) {
                check32(K[c]);
                P.segs.push_back((int32_t)K[c]);            // klen
                P.segs.push_back(0);                        // window over the K half
                P.segs.push_back((int32_t)ceil2(K[c]));
                for (const auto* list : {&pr.x, &pr.y})
                    for (const XTerm& u : *list) {
                        check32(u.rvend[c]);
                        P.segs.push_back((int32_t)u.row[c]);
                        P.segs.push_back((int32_t)u.rvend[c]);
                    }
            }
            if (direct) {
                t.dst = 0;
                t.beta = beta;
                t.dM = (int32_t)M;
                t.dN = (int32_t)N;
                t.r0 = (int32_t)xc;
                t.q0 = (int32_t)yc;
            } else {
                t.dst = 1;
                t.beta = 0;
                t.dM = (int32_t)Mp;
                t.dN = (int32_t)Np;
                t.ws_off = ws_base + (int64_t)s * Mp * Np;
            }
            t.tiles_m = (int32_t)((MHin + kStrTile - 1) / kStrTile);
            t.tiles_n = (int32_t)((NHin + kStrTile - 1) / kStrTile);
            P.mults += 7 * MHin * NHin * khalf;
            P.str_mults += 7 * MHin * NHin * khalf;
            const int32_t id = (int32_t)P.tasks.size();
            P.tasks.push_back(t);
            for (int32_t a = 0; a < t.tiles_m; ++a)
                for (int32_t b = 0; b < t.tiles_n; ++b) ph(gphase).str_items.push_back(WorkItem{id, a, b, 0});
            ph(gphase).str_tmax = std::max(ph(gphase).str_tmax, std::max(t.nx, t.ny));
            ++P.str_tasks;
        }
        if (!direct) {
            DevCombine cb{};
            cb.M = (int32_t)M;
            cb.N = (int32_t)N;
            cb.levels = expand;
            cb.variant = o.variant;
            cb.r0 = (int32_t)xc;
            cb.q0 = (int32_t)yc;
            cb.beta = beta;
            cb.Mp = (int32_t)Mp;
            cb.Np = (int32_t)Np;
            cb.nparts = 1;
            cb.lower = 0;
            cb.part_stride = 0;
            cb.ws_off = ws_base;
            Phase& pz = ph(gphase);
            cb.elem_off = pz.combine_elems;
            pz.combine_elems += M * N;
            P.combine_elems += M * N;
            pz.combines.push_back(cb);
            ++P.combine_tasks;
        }
    }
    return phase + gi;
}

// Window lengths of a task's segments (rows of K each covers).
int64_t task_k(const Plan& P, const DevTask& t) {
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    int64_t k = 0;
    for (int s = 0; s < t.nseg; ++s) k += P.segs[t.seg_off + s * stride + 2] - P.segs[t.seg_off + s * stride + 1];
    return k;
}

// Copy of task t restricted to the k range [a, b) of its concatenated windows.
void restrict_window(Plan& P, DevTask& t, int64_t a, int64_t b) {
    const int stride = kSegHdr + 2 * (t.nx + t.ny);
    std::vector<int32_t> out;
    int nseg = 0;
    int64_t pos = 0;
    for (int s = 0; s < t.nseg; ++s) {
        const int32_t* sg = &P.segs[t.seg_off + s * stride];
        const int64_t w0 = sg[1], w1 = sg[2], len = w1 - w0;
        const int64_t lo = std::max(a, pos), hi = std::min(b, pos + len);
        if (hi > lo) {
            std::vector<int32_t> seg(sg, sg + stride);
            seg[1] = (int32_t)(w0 + (lo - pos));
            seg[2] = (int32_t)(w0 + (hi - pos));
            out.insert(out.end(), seg.begin(), seg.end());
            ++nseg;
        }
        pos += len;
    }
    t.seg_off = (int32_t)P.segs.size();
    t.nseg = nseg;
    P.segs.insert(P.segs.end(), out.begin(), out.end());
}

constexpr int64_t kSplitAlign = 16;

// Resident workgroups of a one-term tile launch in the given split_tail mode.
int64_t tail_slots(int mode) { return mode == 3 ? kTileSlots / 2 : kTileSlots; }

// The one-term classical list of a phase whose short last round the plan
// splits (PlanOptions::split_tail), or null.  Before the mixed lists are
// built (mix_built false) an FP64 phase qualifies by what its mixed list
// will hold.
std::vector<WorkItem>* tail_list(const PlanOptions& o, Phase& ph, bool mix_built) {
    if (o.split_tail == 1) {
        if (ph.tg_tmax > 1) return nullptr;
        if (mix_built) return ph.mix_items.empty() ? nullptr : &ph.mix_items;
        const bool any = !(ph.tg_items.empty() && ph.gemm_items.empty() && ph.syrk_items.empty());
        return ph.str_items.empty() && any ? &ph.mix_items : nullptr;
    }
    if (o.split_tail >= 2 && ph.str_items.empty() && ph.tg_items.empty()) {
        if (ph.gemm_items.empty() && !ph.syrk_items.empty()) return &ph.syrk_items;
        if (ph.syrk_items.empty() && !ph.gemm_items.empty()) return &ph.gemm_items;
    }
    return nullptr;
}

// Split long K ranges of launches that have too few tiles to fill the GPU.
// A task writing C becomes nparts tasks writing dense partial blocks to the
// workspace plus a combination that sums them (in part order) into C; the
// products of a block already written to the workspace get nparts slot sets
// and their combination sums over parts as well.  The scalar products are
// unchanged; only the order of summation over K differs.
void split_k(Plan& P) {
    const PlanOptions& o = P.opt;
    if (o.split_target <= 0) return;
    for (size_t pi = 0; pi < P.phases.size(); ++pi) {
        Phase& ph = P.phases[pi];
        const int64_t items = (int64_t)(ph.str_items.size() + ph.tg_items.size() + ph.gemm_items.size() + ph.syrk_items.size());
        if (items == 0 || items >= o.split_target) continue;
        // launches of more than one round of tiles leave only a last round
        // to balance, which the split of that round does without partials
        // of every tile
        if (items > tail_slots(o.split_tail) && tail_list(o, ph, false)) continue;
        int64_t want = std::min<int64_t>(64, o.split_target / items);
        if (want < 2) continue;
        if ((o.split_tail == 1 || o.split_tail == 2) && ph.str_items.empty() && ph.tg_items.empty()) {
            // classical tiles alone (items of equal cost per unit of K): every
            // part writes a partial tile and the sum reads it back, so take
            // the fewest parts whose rounds of the resident workgroups come
            // within half a percent of the best tile time up to `want` parts
            auto rounds = [&](int64_t p) {
                return (double)((items * p + kTileSlots - 1) / kTileSlots) / (double)p;
            };
            double best = rounds(want);
            for (int64_t p = 2; p < want; ++p) best = std::min(best, rounds(p));
            for (int64_t p = 2; p <= want; ++p)
                if (rounds(p) <= best * 1.005) {
                    want = p;
                    break;
                }
        }
        // decide a part count per task (workspace blocks: per combine block)
        std::map<int32_t, int> parts;  // task id -> parts
        auto decide = [&](int32_t id) {
            if (parts.count(id)) return;
            const int64_t k = task_k(P, P.tasks[id]);
            parts[id] = (int)std::max<int64_t>(1, std::min<int64_t>(want, k / o.split_min_k));
        };
        for (auto* items_v : {&ph.str_items, &ph.tg_items, &ph.gemm_items, &ph.syrk_items})
            for (const WorkItem& w : *items_v) decide(w.task);
        // products of one workspace block must share the part count
        for (DevCombine& cb : ph.combines) {
            int np = 64;
            const int64_t span = (int64_t)cb.Mp * cb.Np * [&] { int p = 1; for (int l = 0; l < cb.levels; ++l) p *= 7; return p; }();
            for (auto& kv : parts) {
                const DevTask& t = P.tasks[kv.first];
                if (t.dst == 1 && t.ws_off >= cb.ws_off && t.ws_off < cb.ws_off + span) np = std::min(np, kv.second);
            }
            for (auto& kv : parts) {
                const DevTask& t = P.tasks[kv.first];
                if (t.dst == 1 && t.ws_off >= cb.ws_off && t.ws_off < cb.ws_off + span) kv.second = np;
            }
            if (np > 1) {
                // fresh workspace for np slot sets; the first keeps the old offset range
                const int64_t base = P.ws_elems;
                P.ws_elems += span * np;
                for (auto& kv : parts) {
                    DevTask& t = P.tasks[kv.first];
                    if (t.dst == 1 && t.ws_off >= cb.ws_off && t.ws_off < cb.ws_off + span)
                        t.ws_off = base + (t.ws_off - cb.ws_off);
                }
                cb.ws_off = base;
                cb.nparts = np;
                cb.part_stride = span;
            }
        }
        // rewrite the tasks and their work items
        std::map<int32_t, std::vector<int32_t>> newids;  // task -> part task ids
        std::map<int32_t, int64_t> stride_of;             // part stride of workspace tasks
        for (auto& kv : parts) {
            const int32_t id = kv.first;
            const int np = kv.second;
            if (np < 2) continue;
            const DevTask t0 = P.tasks[id];
            const int64_t k = task_k(P, t0);
            int64_t pstride = 0;
            int64_t wbase = 0;
            if (t0.dst == 0) {
                // partial blocks written densely, then summed into C
                pstride = (int64_t)t0.dM * t0.N;
                wbase = P.ws_elems;
                P.ws_elems += pstride * np;
                DevCombine cb{};
                cb.M = t0.dM;
                cb.N = t0.dN;
                cb.levels = 0;
                cb.variant = 0;
                cb.r0 = t0.r0;
                cb.q0 = t0.q0;
                cb.beta = t0.beta;
                cb.Mp = t0.dM;
                cb.Np = t0.N;
                cb.nparts = np;
                cb.lower = t0.kind == TK_SYRK ? 1 : 0;
                cb.part_stride = pstride;
                cb.ws_off = wbase;
                cb.elem_off = ph.combine_elems;
                ph.combine_elems += (int64_t)t0.dM * t0.dN;
                ph.combines.push_back(cb);
                ++P.combine_tasks;
            } else {
                for (const DevCombine& cb : ph.combines)
                    if (cb.nparts == np && t0.ws_off >= cb.ws_off && t0.ws_off < cb.ws_off + cb.part_stride)
                        pstride = cb.part_stride;
            }
            // interior part boundaries on multiples of kSplitAlign rows, so that
            // windows stay aligned wherever the row chunks are (the reduced-
            // precision tiles stage whole dwords of a converted copy)
            auto cut = [&](int p) -> int64_t { return p == np ? k : (k * p / np) / kSplitAlign * kSplitAlign; };
            for (int p = 0; p < np; ++p) {
                DevTask t = t0;
                restrict_window(P, t, cut(p), cut(p + 1));
                if (t0.dst == 0) {
                    t.dst = 1;
                    t.beta = 0;
                    t.ws_off = wbase + p * pstride;
                } else {
                    t.ws_off = t0.ws_off + p * pstride;
                }
                const int32_t nid = (int32_t)P.tasks.size();
                newids[id].push_back(nid);
                P.tasks.push_back(t);
                P.task_group.resize(P.tasks.size(), -1);
                P.task_part.resize(P.tasks.size(), 0);
                P.task_group[nid] = P.task_group[id];
                P.task_part[nid] = p;
            }
        }
        for (auto* items_v : {&ph.str_items, &ph.tg_items, &ph.gemm_items, &ph.syrk_items}) {
            std::vector<WorkItem> out;
            for (const WorkItem& w : *items_v) {
                auto it = newids.find(w.task);
                if (it == newids.end()) {
                    out.push_back(w);
                    continue;
                }
                for (int32_t nid : it->second) out.push_back(WorkItem{nid, w.ti, w.tj, w.slot});
            }
            items_v->swap(out);
        }
        // combination blocks ordered by element offset
        std::sort(ph.combines.begin(), ph.combines.end(),
                  [](const DevCombine& a, const DevCombine& b) { return a.elem_off < b.elem_off; });
    }
}

// The classical tasks of a reduced-precision phase on 256 x 256 workgroup
// tiles (k_lp8_big), longest K first, then by tile position.
std::vector<WorkItem> big_tile_items(const Plan& P, const Phase& ph) {
    std::vector<int32_t> ids;
    for (const auto* v : {&ph.gemm_items, &ph.syrk_items})
        for (const WorkItem& w : *v) ids.push_back(w.task);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    std::vector<std::pair<int64_t, WorkItem>> out;
    for (int32_t id : ids) {
        const DevTask& t = P.tasks[id];
        int64_t k = 0;
        const int stride = kSegHdr + 2 * (t.nx + t.ny);
        for (int sg = 0; sg < t.nseg; ++sg) {
            const int32_t* g = P.segs.data() + t.seg_off + (int64_t)sg * stride;
            k += g[2] - g[1];
        }
        const int tm = (t.dM + kBigTile - 1) / kBigTile, tn = (t.dN + kBigTile - 1) / kBigTile;
        for (int a = 0; a < tm; ++a)
            for (int b = 0; b < tn; ++b)
                if (t.kind != TK_SYRK || b <= a) out.push_back({k, WorkItem{id, a, b, 0}});
    }
    // blocks of 4 x 8 tile positions: the 32 workgroups one XCD holds at a
    // time read 4 row panels and 8 column panels between them
    std::stable_sort(out.begin(), out.end(), [](const std::pair<int64_t, WorkItem>& x, const std::pair<int64_t, WorkItem>& y) {
        if (x.first != y.first) return x.first > y.first;
        if (x.second.task != y.second.task) return x.second.task < y.second.task;
        if (x.second.ti / 4 != y.second.ti / 4) return x.second.ti / 4 < y.second.ti / 4;
        if (x.second.tj / 8 != y.second.tj / 8) return x.second.tj / 8 < y.second.tj / 8;
        if (x.second.ti != y.second.ti) return x.second.ti < y.second.ti;
        return x.second.tj < y.second.tj;
    });
    // workgroup 8 j + x runs on XCD x: runs of 32 consecutive items go to the
    // positions of one XCD (a short last round uses shorter runs)
    std::vector<WorkItem> items(out.size());
    size_t base = 0;
    while (base < out.size()) {
        const size_t rem = out.size() - base;
        const size_t run = rem >= 256 ? 32 : rem / 8;
        if (run == 0) {
            for (size_t k = base; k < out.size(); ++k) items[k] = out[k].second;
            break;
        }
        for (size_t c = 0; c < 8; ++c)
            for (size_t j = 0; j < run; ++j) items[base + j * 8 + c] = out[base + c * run + j].second;
        base += 8 * run;
    }
    return items;
}

// Reduced-precision plans: the 256 x 256 e4m3 tiles of every phase.  When
// their count leaves a last round of at most half the resident workgroups,
// those last tiles (the last positions of the launch) become a launch of
// their own with the K range of each split into parts, so that the round
// spreads over every CU; the parts' FP32 results go to the workspace and are
// summed in part order.
void lp_big_tiles(Plan& P) {
    int64_t most = 0;
    for (Phase& ph : P.phases) {
        ph.big_items = big_tile_items(P, ph);
        const int64_t nb = (int64_t)ph.big_items.size(), r = nb % kBigMinTiles;
        if (nb <= kBigMinTiles || r == 0 || r > kBigMinTiles / 2) continue;
        int parts = (int)(kBigMinTiles / r);
        for (int64_t q = nb - r; q < nb; ++q) {
            const DevTask& t = P.tasks[ph.big_items[q].task];
            const int64_t stages = (task_k(P, t) + 127) / 128;
            parts = (int)std::min<int64_t>(parts, stages / 4);
        }
        if (parts < 2) continue;
        for (int64_t q = nb - r; q < nb; ++q)
            for (int p = 0; p < parts; ++p) {
                WorkItem w = ph.big_items[q];
                w.slot = (int32_t)((q - (nb - r)) * parts + p);
                ph.big_tail.push_back(w);
            }
        ph.big_items.resize(nb - r);
        ph.big_tail_parts = parts;
        most = std::max<int64_t>(most, r * parts);
    }
    if (most > 0) {
        P.lp_tail_off = P.ws_elems;
        P.ws_elems += most * kBigTile * kBigTile / 2;  // FP32 partial tiles in FP64 elements
    }
}

// One-term tile launches (classical tiles alone, run one workgroup per
// item) of more than one round: the r items of the last round (the last
// positions of the launch, the shortest in longest-first order) become a
// launch of their own with each tile's K range split into p parts, written
// to the workspace and summed in part order.  The round then takes
// ceil(r p / slots) / p of a tile time instead of one: p = slots / r when r
// is at most half the slots (one round of parts), else the smallest p of at
// most 8 within 0.05 tile times of the best, taken when it saves at least a
// fifth of a tile time.  Every part keeps at least eight 16-row stages.
void split_tail_rounds(Plan& P) {
    int64_t most = 0;
    const int64_t slots = tail_slots(P.opt.split_tail);
    for (Phase& ph : P.phases) {
        std::vector<WorkItem>* list = tail_list(P.opt, ph, true);
        if (!list) continue;
        std::vector<WorkItem>& items = *list;
        const int64_t n = (int64_t)items.size(), r = n % slots;
        if (n <= slots || r == 0) continue;
        int64_t pk = 64;
        for (int64_t q = n - r; q < n; ++q) pk = std::min<int64_t>(pk, task_k(P, P.tasks[items[q].task]) / 128);
        auto cost = [&](int64_t p) { return (double)((r * p + slots - 1) / slots) / (double)p; };
        int parts = 1;
        if (2 * r <= slots) {
            parts = (int)std::min<int64_t>(slots / r, pk);
        } else {
            double best = 1.0;
            for (int64_t p = 2; p <= std::min<int64_t>(8, pk); ++p) best = std::min(best, cost(p));
            for (int64_t p = 2; p <= std::min<int64_t>(8, pk); ++p)
                if (cost(p) <= best + 0.05) {
                    parts = (int)p;
                    break;
                }
            if (parts > 1 && cost(parts) > 0.8) parts = 1;
        }
        if (parts < 2) continue;
        for (int64_t q = n - r; q < n; ++q)
            for (int p = 0; p < parts; ++p) {
                WorkItem w = items[q];
                w.slot = (int32_t)((q - (n - r)) * parts + p);
                ph.tail_items.push_back(w);
            }
        items.resize(n - r);
        ph.tail_parts = parts;
        most = std::max<int64_t>(most, r * parts);
    }
    if (most > 0) {
        P.tile_tail_off = P.ws_elems;
        P.ws_elems += most * kGemmTile * kGemmTile;
    }
}

}  // namespace

Plan build_plan(int64_t m, int64_t n, const PlanOptions& opt) {
    if (m < 0 || n < 0) throw std::invalid_argument("negative dimension");
    if (opt.cutoff < 1) throw std::invalid_argument("cutoff must be positive");
    if (opt.variant != 0 && opt.variant != 1) throw std::invalid_argument("bad variant");
    check32(m);
    check32(n);
    Plan P;
    P.m = m;
    P.n = n;
    P.opt = opt;
    if (m > 0 && n > 0) {
        Builder b(P);
        b.ata_node({Chunk{0, m}}, 0, n, 0, 0);
    }
    split_k(P);
    if (opt.accumulate) {
        for (DevTask& t : P.tasks)
            if (t.dst == 0) t.beta = 1;
        for (Phase& ph : P.phases)
            for (DevCombine& cb : ph.combines) cb.beta = 1;
    }
    // Order of the items of every launch.  Heavier tiles first (longest
    // processing time).  Among equal costs, tiles that read the same operand
    // strips go together: the products of one Strassen expansion (same K
    // part) at neighbouring tile positions, in blocks of B x B positions with
    // B^2 times the product count near 64; classical tiles of one task in
    // 8 x 8 blocks.
    auto group_of = [&](int32_t id) -> int64_t {
        const int32_t g = (size_t)id < P.task_group.size() ? P.task_group[id] : -1;
        return g >= 0 ? ((int64_t)1 << 40) + g : (int64_t)id;
    };
    auto part_of = [&](int32_t id) -> int32_t { return (size_t)id < P.task_part.size() ? P.task_part[id] : 0; };
    std::map<int64_t, int> group_size;  // products per expansion group
    for (size_t id = 0; id < P.tasks.size(); ++id)
        if (part_of((int32_t)id) == 0 && group_of((int32_t)id) >= ((int64_t)1 << 40)) ++group_size[group_of((int32_t)id)];
    auto block_of = [&](int32_t id) -> int {
        const int64_t gk = group_of(id);
        if (gk < ((int64_t)1 << 40)) return 8;
        const int np = std::max(1, group_size[gk]);
        int b = 1;
        while ((b + 1) * (b + 1) * np <= 64) ++b;
        return b;
    };
    for (Phase& ph : P.phases) {
        auto cost = [&](const WorkItem& w) {
            const DevTask& t = P.tasks[w.task];
            const double k = (double)task_k(P, t);
            if (t.kind == TK_STR) return 2.0 * k * (1.0 + 0.1 * (t.nx + t.ny));
            return k * (1.0 + 0.1 * (t.nx + t.ny - 2));
        };
        if (ph.str_items.empty() && ph.tg_tmax <= 2 &&
            !(ph.tg_items.empty() && ph.gemm_items.empty() && ph.syrk_items.empty())) {
            ph.mix_items = ph.tg_items;
            ph.mix_items.insert(ph.mix_items.end(), ph.gemm_items.begin(), ph.gemm_items.end());
            ph.mix_items.insert(ph.mix_items.end(), ph.syrk_items.begin(), ph.syrk_items.end());
        }
        for (auto* items : {&ph.str_items, &ph.tg_items, &ph.gemm_items, &ph.syrk_items, &ph.mix_items})
            std::stable_sort(items->begin(), items->end(), [&](const WorkItem& a, const WorkItem& b) {
                const double ca = cost(a), cb = cost(b);
                if (ca != cb) return ca > cb;
                const int64_t ga = group_of(a.task), gb = group_of(b.task);
                if (ga != gb) return ga < gb;
                const int32_t pa = part_of(a.task), pb = part_of(b.task);
                if (pa != pb) return pa < pb;
                const int B = block_of(a.task);
                if (a.ti / B != b.ti / B) return a.ti / B < b.ti / B;
                if (a.tj / B != b.tj / B) return a.tj / B < b.tj / B;
                if (a.task != b.task) return a.task < b.task;
                if (a.ti != b.ti) return a.ti < b.ti;
                return a.tj < b.tj;
            });
        // Workgroups are dispatched round-robin over the eight XCDs, each with
        // its own L2: item 8 j + x runs on XCD x.  Runs of 64 consecutive
        // items of the order above (about what one XCD holds at a time, two
        // workgroups on each of its 32 CUs) are placed at the positions of
        // one XCD; a short last round uses shorter runs.
        for (auto* items : {&ph.str_items, &ph.tg_items, &ph.gemm_items, &ph.syrk_items, &ph.mix_items}) {
            std::vector<WorkItem>& v = *items;
            std::vector<WorkItem> out(v.size());
            size_t base = 0;
            while (base < v.size()) {
                const size_t rem = v.size() - base;
                const size_t run = rem >= 512 ? 64 : rem / 8;
                if (run == 0) {
                    std::copy(v.begin() + base, v.end(), out.begin() + base);
                    break;
                }
                for (size_t c = 0; c < 8; ++c)
                    for (size_t j = 0; j < run; ++j) out[base + j * 8 + c] = v[base + c * run + j];
                base += 8 * run;
            }
            v.swap(out);
        }
        P.work_items += (int64_t)(ph.str_items.size() + ph.tg_items.size() + ph.gemm_items.size() + ph.syrk_items.size());
    }
    if (opt.lp) lp_big_tiles(P);
    if (opt.split_tail && opt.split_target > 0) split_tail_rounds(P);
    for (const Phase& ph : P.phases)
        if (ph.tg_tmax == 2 && (!ph.mix_items.empty() || !ph.tg_items.empty())) {
            P.queue_off = P.ws_elems;
            P.ws_elems += (kTileQueues + 1) / 2;  // int32 queues in FP64 elements
            break;
        }
    return P;
}

}  // namespace atalib
