// Planner: cut -> per-block programs -> tree levels -> fused passes.
//
// * Crossing gates (Section 2, "cross-block" CZ; iSWAP by Eq. (4way)) are
//   ordered by (cycle, smaller qubit); a CZ takes one path bit, an iSWAP
//   two, and the first crossing gate the highest bits, so an aligned block of
//   path ids shares a prefix (Section 2: x = x_p + x_b, processes spawned
//   per x_p-bit prefix).
// * Each block's program is cut into segments at the cycles holding
//   crossing gates.  Segment l starts with the branch operators of level l
//   (P_s on the block-A endpoint, Z^s on the block-B endpoint of a CZ,
//   Section 2, Eq. (CZ); projector plus per-path flip on both endpoints of
//   an iSWAP); everything between two such cycles is shared by all paths
//   with the same prefix (the checkpoint/branch scheme of Section 2).
// * A segment is split into passes: each pass may apply non-diagonal gates
//   only to qubits held in lane bits or in its R register bits; diagonal
//   gates join any pass once their qubits' earlier gates are scheduled and
//   are merged into as few bitmask groups as possible (Section 2:
//   clustering gates of a kind with reordering; bitmask + mod-8 evaluation
//   of all diagonal gates in one pass).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sf_host.hpp"

namespace sf {

static int popcount64(uint64_t x) { return __builtin_popcountll(x); }

namespace {
void gate2x2(uint8_t kind, std::complex<double> g[4]);
}  // namespace

// <x_T| V |x_T with the S bits replaced by y> for the ops `rest` (V, in order) on the qubits of
// tmask, as a [2^|T|][2^|S|] table; V is multiplied out exactly with the normalised gates.
static std::vector<std::complex<double>> fold_table(const std::vector<HalfOp> &rest, uint32_t tmask, uint32_t smask)
{
    const int n_s = __builtin_popcount(smask);
    int tpos[32], spos[32];
    for (int t = 0, a = 0, b = 0; t < 32; ++t) {
        tpos[t] = ((tmask >> t) & 1) ? a++ : -1;
        spos[t] = ((smask >> t) & 1) ? b++ : -1;
    }
    // V as a 2^n_t x 2^n_t matrix, column by column
    const int D = 1 << __builtin_popcount(tmask);
    std::vector<std::complex<double>> M((size_t)D * D);
    const std::complex<double> omega(std::cos(M_PI / 4), std::sin(M_PI / 4));
    const std::complex<double> s_h(1.0 / std::sqrt(2.0), 0.0), s_xy(0.5, 0.5);
    for (int col = 0; col < D; ++col) {
        std::vector<std::complex<double>> v(D, 0.0);
        v[col] = 1.0;
        for (const HalfOp &op : rest) {
            const int a = tpos[op.q0];
            if (op.kind == HK_T) {
                for (int r = 0; r < D; ++r) if ((r >> a) & 1) v[r] *= omega;
            } else if (op.kind == HK_CZ) {
                const int b = tpos[op.q1];
                for (int r = 0; r < D; ++r) if (((r >> a) & 1) && ((r >> b) & 1)) v[r] = -v[r];
            } else if (op.kind == HK_ISWAP) {
                const int b = tpos[op.q1];
                const std::complex<double> I(0.0, 1.0);
                for (int r = 0; r < D; ++r)
                    if (!((r >> a) & 1) && ((r >> b) & 1)) {
                        const int r2 = r ^ (1 << a) ^ (1 << b);
                        const std::complex<double> x = v[r], y = v[r2];
                        v[r] = I * y;
                        v[r2] = I * x;
                    }
            } else {
                std::complex<double> g[4];
                gate2x2(op.kind, g);
                const std::complex<double> sc = op.kind == HK_H ? s_h : s_xy;
                for (int r = 0; r < D; ++r) {
                    if ((r >> a) & 1) continue;
                    const int r1 = r | (1 << a);
                    const std::complex<double> x0 = v[r], x1 = v[r1];
                    v[r] = sc * (g[0] * x0 + g[1] * x1);
                    v[r1] = sc * (g[2] * x0 + g[3] * x1);
                }
            }
        }
        for (int r = 0; r < D; ++r) M[(size_t)r * D + col] = v[r];
    }
    // table row x_T, entry y: column = x_T with its S bits replaced by y
    std::vector<std::complex<double>> tab((size_t)D << n_s, 0.0);
    for (int xt = 0; xt < D; ++xt)
        for (int y = 0; y < (1 << n_s); ++y) {
            int col = xt;
            for (int t = 0; t < 32; ++t)
                if (spos[t] >= 0) {
                    const int bit = (y >> spos[t]) & 1;
                    col = (col & ~(1 << tpos[t])) | (bit << tpos[t]);
                }
            tab[((size_t)xt << n_s) + y] = M[(size_t)xt * D + col];
        }
    return tab;
}

static LeafFold make_fold_iswap(const Circuit &c, int h, int F);

// The last F tree levels of block h as V * D(b) (see LeafFold).  Their segments, in order, are
// applied to the state of the level above; the branch operators are diagonal, so each one can
// be moved to the right of every earlier gate of these segments that is diagonal or acts on
// other qubits.  The form holds when no non-diagonal gate precedes a branch operator on its
// qubit, and it is used when every non-diagonal gate of the segments acts on a branch qubit
// (then a descendant reads no more rows of the level above than it has branch values).  V is
// multiplied out exactly with the normalised gates.
static LeafFold make_fold(const Circuit &c, int h, int F)
{
    LeafFold f;
    const int L = (int)c.levels.size() - 1;
    if (F < 1 || F > L) return f;
    for (int l = L - F + 1; l <= L; ++l)
        for (const HalfOp &op : c.half[h].segments[l])
            if (op.kind == HK_PFLIP || op.kind == HK_PFLIPI) return make_fold_iswap(c, h, F);
    const int nb = c.k - c.levels[L - F].bits_after;     // path bits decided by the F levels
    if (nb < 1 || nb > kMaxFoldBits) return f;
    int bq[kMaxFoldBits];
    for (int u = 0; u < kMaxFoldBits; ++u) bq[u] = -1;  // local qubit of the branch operator of path bit u
    uint32_t nondiag_seen = 0, smask = 0, tmask = 0;
    std::vector<HalfOp> rest;
    for (int l = L - F + 1; l <= L; ++l)
        for (const HalfOp &op : c.half[h].segments[l]) {
            if (op.kind == HK_PROJ || op.kind == HK_ZCTL) {
                if (op.bit >= nb || bq[op.bit] >= 0 || op.q0 >= 32 || ((nondiag_seen >> op.q0) & 1)) return f;
                bq[op.bit] = op.q0;
                continue;
            }
            if (op.q0 >= 32 || (is_two_qubit(op.kind) && op.q1 >= 32)) return f;
            const uint32_t om = (1u << op.q0) | (is_two_qubit(op.kind) ? 1u << op.q1 : 0u);
            if (!is_diag(op.kind)) {
                nondiag_seen |= om;
                smask |= om;
            }
            tmask |= om;
            rest.push_back(op);
        }
    uint32_t bmask = 0;
    for (int u = 0; u < nb; ++u) {
        if (bq[u] < 0) return f;
        bmask |= 1u << bq[u];
    }
    f.levels = F;
    f.nb = nb;
    for (int u = 0; u < nb; ++u) f.bq[u] = bq[u];
    // general form: every branch qubit joins S (an identity there), so each column pattern's
    // branch bits are the descendant's branch values
    const uint32_t gs = smask | bmask, gt = tmask | bmask;
    const int gns = __builtin_popcount(gs), gnt = __builtin_popcount(gt);
    if (nb <= kMaxGeneralFoldBits && __builtin_popcount(bmask) == nb && gns <= kMaxGeneralFoldS &&
        gns + gnt <= kMaxGeneralFoldTableBits) {
        const std::vector<std::complex<double>> std_tab = fold_table(rest, gt, gs);
        int gpos[32];                                    // index of each S' qubit in ascending order
        for (int t = 0, b = 0; t < 32; ++t) gpos[t] = ((gs >> t) & 1) ? b++ : -1;
        int col_q[32];                                   // qubit of column bit i
        for (int u = 0; u < nb; ++u) col_q[u] = bq[u];
        for (int t = 0, i = nb; t < 32; ++t)
            if (((gs & ~bmask) >> t) & 1) col_q[i++] = t;
        const int D = 1 << gns;
        f.goff.assign(D, 0);
        std::vector<int> ystd(D, 0);
        for (int y = 0; y < D; ++y)
            for (int i = 0; i < gns; ++i)
                if ((y >> i) & 1) {
                    f.goff[y] |= 1u << col_q[i];
                    ystd[y] |= 1 << gpos[col_q[i]];
                }
        f.gtab.assign((size_t)1 << (gnt + gns), 0.0);
        for (int xt = 0; xt < (1 << gnt); ++xt)
            for (int y = 0; y < D; ++y) f.gtab[((size_t)xt << gns) + y] = std_tab[((size_t)xt << gns) + ystd[y]];
        f.g_ns = gns;
        f.g_nt = gnt;
        f.g_smask = gs;
        f.g_tmask = gt;
        f.gen_ok = true;
    }
    if ((smask & ~bmask) != 0) return f;            // a non-diagonal gate off the branch qubits
    const int n_t = __builtin_popcount(tmask), n_s = __builtin_popcount(smask);
    if (n_t > 8) return f;
    f.tab = fold_table(rest, tmask, smask);
    int spos[32];
    for (int t = 0, b = 0; t < 32; ++t) spos[t] = ((smask >> t) & 1) ? b++ : -1;
    for (int u = 0; u < nb; ++u) {
        f.bq[u] = bq[u];
        f.ypos[u] = spos[bq[u]];
    }
    f.levels = F;
    f.nb = nb;
    f.n_s = n_s;
    f.n_t = n_t;
    f.smask = smask;
    f.tmask = tmask;
    f.dmask = bmask & ~smask;
    f.ok = true;
    return f;
}

// The last F tree levels of block h when all their crossing gates are iSWAPs.  Gate g's branch
// operators on this block are a projector and a per-path flip on one qubit (X^{i xor j} P_j on
// block A, i^{i xor j} X^{i xor j} P_i on block B; the factor i^{i xor j} is left to the kernel).
// The form holds when they are the first operations on their qubit within these levels; every
// other operation is part of V, and every non-diagonal one must act on a gate qubit.
static LeafFold make_fold_iswap(const Circuit &c, int h, int F)
{
    LeafFold f;
    const int L = (int)c.levels.size() - 1;
    const int nb = c.k - c.levels[L - F].bits_after;
    if (nb < 2 || nb > 2 * kMaxFoldGates || (nb & 1)) return f;
    int proj_bit[32];
    for (int q = 0; q < 32; ++q) proj_bit[q] = -1;        // PROJ seen, its flip not yet
    uint32_t seen = 0, covered = 0, qmask = 0, smask = 0, tmask = 0;
    int ng = 0, gq[kMaxFoldGates], gu[kMaxFoldGates];
    std::vector<HalfOp> rest;
    for (int l = L - F + 1; l <= L; ++l)
        for (const HalfOp &op : c.half[h].segments[l]) {
            if (op.q0 >= 32 || (is_two_qubit(op.kind) && op.q1 >= 32)) return f;
            const uint32_t m0 = 1u << op.q0;
            if (op.kind == HK_ZCTL) return f;
            if (op.kind == HK_PROJ) {
                if (seen & m0) return f;
                proj_bit[op.q0] = op.bit;
                seen |= m0;
                continue;
            }
            if (op.kind == HK_PFLIP || op.kind == HK_PFLIPI) {
                const int u = op.bit;
                const bool want_b = h == 1;
                if ((op.kind == HK_PFLIPI) != want_b || u + 1 >= nb) return f;
                if (proj_bit[op.q0] != (want_b ? u + 1 : u)) return f;
                if ((covered >> u) & 3u) return f;
                if (ng == kMaxFoldGates) return f;
                covered |= 3u << u;
                qmask |= m0;
                gq[ng] = op.q0;
                gu[ng] = u;
                ++ng;
                proj_bit[op.q0] = -2;
                continue;
            }
            const uint32_t m = m0 | (is_two_qubit(op.kind) ? 1u << op.q1 : 0u);
            for (int q = 0; q < 32; ++q)
                if (((m >> q) & 1) && proj_bit[q] >= 0) return f;   // between a projector and its flip
            if (!is_diag(op.kind)) smask |= m;
            tmask |= m;
            seen |= m;
            rest.push_back(op);
        }
    if (covered != (nb >= 32 ? ~0u : (1u << nb) - 1)) return f;
    if ((smask & ~qmask) != 0) return f;            // a non-diagonal gate off the gate qubits
    const int n_t = __builtin_popcount(tmask);
    if (n_t > 8) return f;
    f.tab = fold_table(rest, tmask, smask);
    int spos[32];
    for (int t = 0, b = 0; t < 32; ++t) spos[t] = ((smask >> t) & 1) ? b++ : -1;
    f.iswap = true;
    f.ng = ng;
    for (int g = 0; g < ng; ++g) {
        f.gq[g] = gq[g];
        f.gu[g] = gu[g];
        f.gy[g] = spos[gq[g]];
    }
    f.qmask = qmask;
    f.levels = F;
    f.nb = nb;
    f.n_s = __builtin_popcount(smask);
    f.n_t = n_t;
    f.smask = smask;
    f.tmask = tmask;
    f.ok = true;
    return f;
}

// The deepest fold whose non-diagonal gates act on branch qubits only, else the deepest general
// one (which reads more rows of the level above per bitstring).
int fold_depth(const Circuit &c)
{
    if (c.tuning.no_leaf_fold) return 0;
    int best = 0, best_gen = 0;
    const int n = (int)std::min(c.half[0].folds.size(), c.half[1].folds.size());
    for (int F = 1; F <= n; ++F) {
        if (c.tuning.fold_levels && F > (int)c.tuning.fold_levels) break;
        const LeafFold &a = c.half[0].folds[F - 1], &b = c.half[1].folds[F - 1];
        if (a.ok && b.ok && a.iswap == b.iswap) best = F;
        if (a.gen_ok && b.gen_ok) best_gen = F;
    }
    return best ? best : best_gen;
}

DeferredLevel deferred_level(const Circuit &c, int h, int level)
{
    DeferredLevel d;
    if (level < 1 || level >= (int)c.half[h].segments.size()) return d;
    const std::complex<double> I(0.0, 1.0), w(std::sqrt(0.5), std::sqrt(0.5));
    int slot_of[64];
    for (int q = 0; q < 64; ++q) slot_of[q] = -1;
    for (const HalfOp &op : c.half[h].segments[level]) {
        if (op.kind == HK_PROJ) {
            // the projector must come first on its qubit, once
            if (slot_of[op.q0] >= 0 || d.n == kMaxDeferredBits) return DeferredLevel();
            const int i = d.n++;
            slot_of[op.q0] = i;
            d.q[i] = op.q0;
            d.u[i] = op.bit;
            d.mask |= 1u << op.q0;
            d.v[i][0][0] = d.v[i][1][1] = 1.0;
            d.v[i][0][1] = d.v[i][1][0] = 0.0;
            continue;
        }
        std::complex<double> g[2][2];
        switch (op.kind) {
        case HK_H: g[0][0] = 1.0; g[0][1] = 1.0; g[1][0] = 1.0; g[1][1] = -1.0; break;
        case HK_X: g[0][0] = 1.0; g[0][1] = -I; g[1][0] = -I; g[1][1] = 1.0; break;
        case HK_Y: g[0][0] = 1.0; g[0][1] = -1.0; g[1][0] = 1.0; g[1][1] = 1.0; break;
        case HK_T: g[0][0] = 1.0; g[0][1] = 0.0; g[1][0] = 0.0; g[1][1] = w; break;
        default: return DeferredLevel();          // two-qubit, other branch operators
        }
        const int i = op.q0 < 64 ? slot_of[op.q0] : -1;
        if (i < 0) return DeferredLevel();        // a gate on a qubit without a projector
        std::complex<double> m[2][2];
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < 2; ++s) m[r][s] = g[r][0] * d.v[i][0][s] + g[r][1] * d.v[i][1][s];
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < 2; ++s) d.v[i][r][s] = m[r][s];
    }
    d.ok = d.n > 0;
    return d;
}

bool fold_general(const Circuit &c, int FD)
{
    if (FD < 1) return false;
    const LeafFold &a = c.half[0].folds[FD - 1], &b = c.half[1].folds[FD - 1];
    return !(a.ok && b.ok && a.iswap == b.iswap);
}

int build_programs(Circuit &c, std::string &err)
{
    const int n = c.n;
    int local[64];
    for (int q = 0; q < n; ++q) {
        const uint64_t m = ((c.mask_a >> q) & 1) ? c.mask_a : c.mask_b;
        local[q] = popcount64(m & ((q ? (uint64_t(1) << q) : 0) - 1));
        if (q == 0) local[q] = 0;
    }
    auto in_a = [&](int q) { return ((c.mask_a >> q) & 1) != 0; };

    // crossing two-qubit gates in path-bit order; a CZ takes one path bit (two terms), an iSWAP
    // two (the four terms of Eq. (4way)), and the first crossing gate the highest bits
    c.cut_gate.clear();
    for (size_t i = 0; i < c.gates.size(); ++i) {
        const sf_gate_t &g = c.gates[i];
        if ((g.kind == 4 || g.kind == 5) && in_a(g.q0) != in_a(g.q1)) c.cut_gate.push_back((int)i);
    }
    std::stable_sort(c.cut_gate.begin(), c.cut_gate.end(), [&](int a, int b) {
        const sf_gate_t &x = c.gates[a], &y = c.gates[b];
        const int mx = std::min(x.q0, x.q1), my = std::min(y.q0, y.q1);
        return x.cycle != y.cycle ? x.cycle < y.cycle : mx < my;
    });
    auto width = [&](int gi) { return c.gates[gi].kind == 5 ? 2 : 1; };
    c.k = 0;
    for (int gi : c.cut_gate) c.k += width(gi);
    if (c.k > 62) {
        err = "crossing gates take more than 62 path bits";
        return SF_ERR_UNSUPPORTED;
    }
    std::vector<int> bit_of_gate(c.gates.size(), -1);   // lowest path bit of the gate's term index
    for (int j = 0, top = c.k; j < (int)c.cut_gate.size(); ++j) {
        top -= width(c.cut_gate[j]);
        bit_of_gate[c.cut_gate[j]] = top;
    }

    // tree levels: one per clock cycle that holds crossing gates
    c.levels.clear();
    c.levels.push_back(Level{-1, 0, 0, 0});
    for (int j = 0; j < (int)c.cut_gate.size(); ++j) {
        const int gi = c.cut_gate[j];
        const int cy = c.gates[gi].cycle;
        if (c.levels.size() == 1 || c.levels.back().cycle != cy)
            c.levels.push_back(Level{cy, j, 0, 0});
        c.levels.back().n_cut += width(gi);
        c.levels.back().bits_after = c.k - bit_of_gate[gi];
    }
    const int L = (int)c.levels.size() - 1;

    for (int h = 0; h < 2; ++h) {
        HalfProgram &hp = c.half[h];
        hp.q = popcount64(h == 0 ? c.mask_a : c.mask_b);
        hp.segments.assign(L + 1, {});
        hp.init_h_mask = 0;
    }
    // Per block, the operations in list order; a crossing gate becomes its branch operators,
    // tagged with its tree level.  Crossing CZ (Section 2, Eq. (CZ)): P_s on the A endpoint,
    // Z^s on the B endpoint.  Crossing iSWAP, term r = 2i + j of Eq. (4way) (i = path bit u+1,
    // j = path bit u): |i><j| = X^{i xor j} P_j on the A endpoint and, by Eq. (iSWAP1),
    // G_ij = i^{i xor j} X^{i xor j} P_i on the B endpoint.
    std::vector<HalfOp> ops[2];
    std::vector<int> own[2];
    for (size_t i = 0; i < c.gates.size(); ++i) {
        const sf_gate_t &g = c.gates[i];
        if (bit_of_gate[i] >= 0) {
            int lvl = 1;
            while (c.levels[lvl].cycle != g.cycle) ++lvl;
            const uint8_t qa = (uint8_t)local[in_a(g.q0) ? g.q0 : g.q1];
            const uint8_t qb = (uint8_t)local[in_a(g.q0) ? g.q1 : g.q0];
            const uint8_t u = (uint8_t)bit_of_gate[i];
            if (g.kind == 4) {
                ops[0].push_back(HalfOp{HK_PROJ, qa, 0, u});
                ops[1].push_back(HalfOp{HK_ZCTL, qb, 0, u});
            } else {
                ops[0].push_back(HalfOp{HK_PROJ, qa, 0, u});
                ops[0].push_back(HalfOp{HK_PFLIP, qa, 0, u});
                ops[1].push_back(HalfOp{HK_PROJ, qb, 0, (uint8_t)(u + 1)});
                ops[1].push_back(HalfOp{HK_PFLIPI, qb, 0, u});
            }
            own[0].resize(ops[0].size(), lvl);
            own[1].resize(ops[1].size(), lvl);
            continue;
        }
        const int h = in_a(g.q0) ? 0 : 1;
        const uint8_t a = (uint8_t)local[g.q0];
        if (g.kind == 5) {
            // iSWAP inside a block: one operation on both qubits (a swap of the |01> and |10>
            // amplitudes, each times i)
            ops[h].push_back(HalfOp{HK_ISWAP, a, (uint8_t)local[g.q1], 0});
            own[h].push_back(0);
            continue;
        }
        HalfOp op{0, a, 0, 0};
        switch (g.kind) {
        case 0: op.kind = HK_H; break;
        case 1: op.kind = HK_X; break;
        case 2: op.kind = HK_Y; break;
        case 3: op.kind = HK_T; break;
        default: op.kind = HK_CZ; op.q1 = (uint8_t)local[g.q1]; break;
        }
        ops[h].push_back(op);
        own[h].push_back(0);
    }
    // Each operation runs at the highest tree level its dependencies allow, so work that does
    // not depend on a level's branch operators is done once per parent instead of once per
    // child.  Diagonal operators commute with each other (and the branch operators are
    // diagonal): a diagonal op waits only for earlier non-diagonal ops on its qubits, a
    // non-diagonal op waits for everything earlier on its qubit.
    for (int h = 0; h < 2; ++h) {
        std::vector<int> N(64, 0), D(64, 0);   // level of the last non-diagonal op / of later diagonal ops
        for (size_t i = 0; i < ops[h].size(); ++i) {
            const HalfOp &op = ops[h][i];
            int lvl = own[h][i];
            if (is_diag(op.kind)) {
                lvl = std::max(lvl, N[op.q0]);
                if (op.kind == HK_CZ) lvl = std::max(lvl, N[op.q1]);
                D[op.q0] = std::max(D[op.q0], lvl);
                if (op.kind == HK_CZ) D[op.q1] = std::max(D[op.q1], lvl);
            } else {
                lvl = std::max(lvl, std::max(N[op.q0], D[op.q0]));
                if (op.kind == HK_ISWAP) lvl = std::max(lvl, std::max(N[op.q1], D[op.q1]));
                N[op.q0] = lvl;
                D[op.q0] = lvl;
                if (op.kind == HK_ISWAP) N[op.q1] = D[op.q1] = lvl;
            }
            c.half[h].segments[lvl].push_back(op);
        }
    }

    // fold each qubit's opening H (if it is the qubit's first operation) into the initial state,
    // then the scalar of the unnormalised gates and the power-of-two rescaling per segment
    const std::complex<double> s_h(1.0 / std::sqrt(2.0), 0.0), s_xy(0.5, 0.5);
    for (int h = 0; h < 2; ++h) {
        HalfProgram &hp = c.half[h];
        uint64_t touched = 0;
        std::vector<HalfOp> kept;
        int folded = 0;
        for (const HalfOp &op : hp.segments[0]) {
            const uint64_t m = (uint64_t(1) << op.q0) | (is_two_qubit(op.kind) ? uint64_t(1) << op.q1 : 0);
            if (op.kind == HK_H && !(touched & m)) {
                hp.init_h_mask |= m;
                ++folded;
                touched |= m;
                continue;
            }
            touched |= m;
            kept.push_back(op);
        }
        hp.segments[0] = kept;
        hp.init_scale = std::pow(s_h, folded);
        hp.seg_scale.assign(L + 1, 1.0);
        hp.seg_rescale_exp.assign(L + 1, 0);
        int carry = 0;
        for (int l = 0; l <= L; ++l) {
            int nh = 0, nxy = 0;
            for (const HalfOp &op : hp.segments[l]) {
                if (op.kind == HK_H) ++nh;
                else if (op.kind == HK_X || op.kind == HK_Y) ++nxy;
            }
            carry += nh + nxy;              // each unnormalised gate multiplies the norm by sqrt2
            const int e = carry / 2;
            carry -= 2 * e;
            hp.seg_rescale_exp[l] = e;
            hp.seg_scale[l] = std::pow(s_h, nh) * std::pow(s_xy, nxy) * std::ldexp(1.0, e);
        }
    }
    c.exec_cache.reset();
    for (int h = 0; h < 2; ++h) {
        c.half[h].folds.clear();
        for (int F = 1; F <= L; ++F) c.half[h].folds.push_back(make_fold(c, h, F));
    }
    c.equal_bits = equal_bit_pairs(c);
    c.plan_cache.clear();
    return SF_OK;
}

// Pairs of path bits that a path with a nonzero term sets equal (Section 2: the projectors of
// the cut gates leave zero blocks in the block states; here the whole state).  Each block's
// program is walked in order, tracking per qubit the path bit whose value the qubit is known to
// hold: a projector onto path bit u sets it (and, if the qubit already holds path bit v, the
// product of the two projectors is zero unless bits u and v are equal); diagonal gates keep it;
// the per-path flip of a crossing iSWAP on bits (u, u+1) swaps u and u+1 (it flips exactly
// when they differ) and otherwise forgets; every other non-diagonal gate forgets it.  Within a
// segment the planner keeps the order of the operations on each qubit.
std::vector<std::pair<int, int>> equal_bit_pairs(const Circuit &c)
{
    std::vector<std::pair<int, int>> pairs;
    for (int h = 0; h < 2; ++h) {
        int held[64];
        for (int q = 0; q < 64; ++q) held[q] = -1;
        for (const std::vector<HalfOp> &seg : c.half[h].segments)
            for (const HalfOp &op : seg) {
                const int t = op.q0;
                if (op.kind == HK_PROJ) {
                    if (held[t] >= 0 && held[t] != op.bit) pairs.push_back({held[t], op.bit});
                    held[t] = op.bit;
                } else if (op.kind == HK_PFLIP || op.kind == HK_PFLIPI) {
                    held[t] = held[t] == op.bit ? op.bit + 1 : held[t] == op.bit + 1 ? op.bit : -1;
                } else if (op.kind == HK_ISWAP) {
                    std::swap(held[t], held[op.q1]);       // |ab> -> (phase) |ba>
                } else if (!is_diag(op.kind)) {
                    held[t] = -1;
                }
            }
    }
    return pairs;
}

bool path_is_live(const Circuit &c, uint64_t id)
{
    for (const auto &pr : c.equal_bits)
        if (((id >> pr.first) ^ (id >> pr.second)) & 1u) return false;
    return true;
}

// ----------------------------------------------------------------------------
// Diagonal group construction
// ----------------------------------------------------------------------------

namespace {

struct PendingDiag {
    std::map<int, int> lin;                        // ext bit -> weight mod 8
    std::vector<std::pair<int, int>> quad;         // ext bit pairs (a < b), XOR set
    std::vector<std::pair<int, int>> zs;           // (ext bit, path bit), XOR set
    std::vector<std::pair<int, int>> proj;         // (ext bit, path bit), set
    uint64_t touched = 0;                          // local qubits
    bool empty() const { return lin.empty() && quad.empty() && zs.empty() && proj.empty(); }
};

void toggle(std::vector<std::pair<int, int>> &v, std::pair<int, int> x)
{
    auto it = std::find(v.begin(), v.end(), x);
    if (it == v.end()) v.push_back(x);
    else v.erase(it);
}

// Emits the group into pp and appends a PO_DIAG op.
void flush(PendingDiag &pd, PassPlan &pp, const int (&kidx)[64])
{
    if (pd.empty()) { pd = PendingDiag(); return; }
    DiagGroup g;
    std::memset(&g, 0, sizeof(g));
    g.term_off = (uint32_t)(pp.terms.size() / 2);
    std::vector<uint8_t> t;
    auto reg = [&](int bit) { return kidx[bit]; };   // -1 if not a register bit
    int tab[64] = {0};
    const int N = 1 << pp.R;
    bool odd = false;      // some weight is not a multiple of 4 (the phase is not a sign)
    // lin
    std::vector<std::pair<int, int>> lin_b;
    for (auto &kv : pd.lin) {
        const int w = kv.second & 7;
        if (!w) continue;
        if (w & 3) odd = true;
        const int k = reg(kv.first);
        if (k >= 0) {
            for (int j = 0; j < N; ++j) if ((j >> k) & 1) tab[j] += w;
        } else {
            lin_b.push_back({kv.first, w});
        }
    }
    std::vector<std::pair<int, int>> qbb, qbr, zsb, zsr, pb, pr;
    for (auto &e : pd.quad) {
        const int ka = reg(e.first), kb = reg(e.second);
        if (ka >= 0 && kb >= 0) {
            for (int j = 0; j < N; ++j) if (((j >> ka) & 1) && ((j >> kb) & 1)) tab[j] += 4;
        } else if (ka < 0 && kb < 0) {
            qbb.push_back(e);
        } else if (ka < 0) {
            qbr.push_back({e.first, kb});
        } else {
            qbr.push_back({e.second, ka});
        }
    }
    for (auto &e : pd.zs) {
        const int k = reg(e.first);
        if (k >= 0) zsr.push_back({k, e.second});
        else zsb.push_back(e);
    }
    for (auto &e : pd.proj) {
        const int k = reg(e.first);
        if (k >= 0) pr.push_back({k, e.second});
        else pb.push_back(e);
    }
    auto put = [&](const std::vector<std::pair<int, int>> &v) {
        for (auto &e : v) { t.push_back((uint8_t)e.first); t.push_back((uint8_t)e.second); }
    };
    put(lin_b); put(qbb); put(qbr); put(zsb); put(zsr); put(pb); put(pr);
    g.n_lin_b = (uint16_t)lin_b.size();
    g.n_quad_bb = (uint16_t)qbb.size();
    g.n_quad_br = (uint16_t)qbr.size();
    g.n_zs_b = (uint16_t)zsb.size();
    g.n_zs_r = (uint16_t)zsr.size();
    g.n_proj_b = (uint16_t)pb.size();
    g.n_proj_r = (uint16_t)pr.size();
    // bits 2 and 3: some register-only weight sum has bit 0 (an odd power of omega) or bit 1
    // (a factor i); without them every register takes the lane's own factor
    bool reg_odd = false, reg_i = false;
    for (int j = 0; j < N; ++j) {
        reg_odd = reg_odd || (tab[j] & 1);
        reg_i = reg_i || (tab[j] & 2);
    }
    g.flags = (odd ? 1u : 0u) | ((pb.size() + pr.size()) ? 2u : 0u) | (reg_odd ? 4u : 0u) | (reg_i ? 8u : 0u);
    for (int j = 0; j < 64; ++j) {
        const uint64_t v = (uint64_t)(tab[j] & 7);
        g.tab[j >> 4] |= v << ((j & 15) * 4);
    }
    if (!zsb.empty() || !zsr.empty() || !pb.empty() || !pr.empty()) pp.needs_slot_path = true;
    pp.terms.insert(pp.terms.end(), t.begin(), t.end());
    PassOp op{PO_DIAG, 0, 0, 0, (uint32_t)pp.groups.size()};
    pp.groups.push_back(g);
    pp.ops.push_back(op);
    pd = PendingDiag();
}

}  // namespace

namespace {

// Unnormalised one-qubit forms (the kernels use the same; the host scalars cover the rest).
void gate2x2(uint8_t kind, std::complex<double> g[4])
{
    const std::complex<double> I(0, 1);
    if (kind == HK_H) { g[0] = 1; g[1] = 1; g[2] = 1; g[3] = -1; }
    else if (kind == HK_X) { g[0] = 1; g[1] = -I; g[2] = -I; g[3] = 1; }
    else { g[0] = 1; g[1] = -1; g[2] = 1; g[3] = 1; }
}

// Dense block: ops (all inside the four block qubits qs, ascending local ids) multiplied into a
// 16 x 16 complex matrix, returned as its 32 x 32 real embedding [[Ur, -Ui], [Ui, Ur]].
std::vector<float> dense_matrix(const std::vector<HalfOp> &ops, const int qs[4])
{
    std::complex<double> M[16][16];
    for (int r = 0; r < 16; ++r)
        for (int c2 = 0; c2 < 16; ++c2) M[r][c2] = r == c2 ? 1.0 : 0.0;
    auto idx = [&](int q) { for (int t = 0; t < 4; ++t) if (qs[t] == q) return t; return -1; };
    const std::complex<double> omega(std::cos(M_PI / 4), std::sin(M_PI / 4));
    for (const HalfOp &op : ops) {
        if (op.kind == HK_T) {
            const int t = idx(op.q0);
            for (int r = 0; r < 16; ++r) if ((r >> t) & 1) for (int c2 = 0; c2 < 16; ++c2) M[r][c2] *= omega;
        } else if (op.kind == HK_CZ) {
            const int t1 = idx(op.q0), t2 = idx(op.q1);
            for (int r = 0; r < 16; ++r) if (((r >> t1) & 1) && ((r >> t2) & 1)) for (int c2 = 0; c2 < 16; ++c2) M[r][c2] = -M[r][c2];
        } else if (op.kind == HK_ISWAP) {
            const int t1 = idx(op.q0), t2 = idx(op.q1);
            const std::complex<double> I(0.0, 1.0);
            for (int r = 0; r < 16; ++r) {
                if (((r >> t1) & 1) || !((r >> t2) & 1)) continue;
                const int r2 = r ^ (1 << t1) ^ (1 << t2);
                for (int c2 = 0; c2 < 16; ++c2) {
                    const std::complex<double> x = M[r][c2], y = M[r2][c2];
                    M[r][c2] = I * y;
                    M[r2][c2] = I * x;
                }
            }
        } else {
            std::complex<double> g[4];
            gate2x2(op.kind, g);
            const int t = idx(op.q0);
            for (int r = 0; r < 16; ++r) {
                if ((r >> t) & 1) continue;
                const int r1 = r | (1 << t);
                for (int c2 = 0; c2 < 16; ++c2) {
                    const std::complex<double> a = M[r][c2], b = M[r1][c2];
                    M[r][c2] = g[0] * a + g[1] * b;
                    M[r1][c2] = g[2] * a + g[3] * b;
                }
            }
        }
    }
    std::vector<float> m(32 * 32);
    for (int i = 0; i < 16; ++i)
        for (int k = 0; k < 16; ++k) {
            m[i * 32 + k] = (float)M[i][k].real();
            m[i * 32 + 16 + k] = (float)-M[i][k].imag();
            m[(16 + i) * 32 + k] = (float)M[i][k].imag();
            m[(16 + i) * 32 + 16 + k] = (float)M[i][k].real();
        }
    return m;
}

}  // namespace

// The passes of one block over tree levels level0..level (usually one level).  max_lq: a pass may
// keep up to this many qubits (0..2) in lane bits 5 and 4 when the slots fill all six lane bits
// (PassArgs::lane_qpos).
static SegmentPlan plan_segment(const Circuit &c, int half, int level0, int level, int p, int R, int dense_m,
                                int max_lq, const std::vector<HalfOp> *prefix = nullptr, int prefix_exp = 0)
{
    const HalfProgram &hp = c.half[half];
    const int q = hp.q;
    const int n_ext = p + q;
    // With fewer than six slot bits the lowest qubits fill the other lane bits; with max_lq = m
    // the top m lane bits are freed for chosen qubits instead (lq, lq4 below), so qubits
    // 0..n_lane_q-1 sit in the fixed lane bits and qubit n_lane_q.. in registers or tile bits.
    const bool lq_small = p < 6 && max_lq >= 1;
    const int n_lane_q = std::max(0, std::min(q, 6 - p - (lq_small ? max_lq : 0)));
    const int n_free = q - std::max(0, std::min(q, 6 - p));
    const int R_eff = std::max(0, std::min({R, n_ext - 6, n_free}));

    SegmentPlan sp;
    std::vector<HalfOp> rem;
    int seg_exp = prefix_exp;
    if (prefix) rem = *prefix;
    for (int l = level0; l <= level; ++l) {
        rem.insert(rem.end(), hp.segments[l].begin(), hp.segments[l].end());
        seg_exp += hp.seg_rescale_exp[l];
    }
    // rescaling inside the segment: keep the running norm gain below 2^16
    int carry = 0;
    for (int l = 0; l < level0; ++l) {
        int nn = 0;
        for (const HalfOp &op : hp.segments[l]) if (has_gain(op.kind)) ++nn;
        carry = (carry + nn) % 2;
    }
    int taken = 0;
    // An iSWAP whose two qubits cannot both sit in one pass (fewer free registers and lane-qubit
    // slots than it needs) is applied as H_b H_a CZ H_a H_b CZ H_b H_a followed by S = T^2 on both
    // qubits, which is the iSWAP exactly; its six unnormalised H gates gain a factor 8, divided
    // out with the segment's rescaling.
    {
        const bool lq_seg = max_lq >= 1 && n_lane_q == 0 && p >= 6 && q > R_eff;   // p < 6: not counted
        const bool lq4_seg = lq_seg && max_lq >= 2 && q > R_eff + 1;
        const int cap = R_eff + (lq_seg ? 1 : 0) + (lq4_seg ? 1 : 0);
        std::vector<HalfOp> out;
        for (const HalfOp &op : rem) {
            if (op.kind == HK_ISWAP && (op.q0 >= n_lane_q) + (op.q1 >= n_lane_q) > cap) {
                const uint8_t a = op.q0, b = op.q1;
                const HalfOp seq[] = {{HK_H, b, 0, 0}, {HK_H, a, 0, 0}, {HK_CZ, a, b, 0}, {HK_H, a, 0, 0},
                                      {HK_H, b, 0, 0}, {HK_CZ, a, b, 0}, {HK_H, b, 0, 0}, {HK_H, a, 0, 0},
                                      {HK_T, a, 0, 0}, {HK_T, a, 0, 0}, {HK_T, b, 0, 0}, {HK_T, b, 0, 0}};
                for (const HalfOp &x : seq) out.push_back(x);
                seg_exp += 3;
                continue;
            }
            out.push_back(op);
        }
        rem.swap(out);
    }

    // Zero subspace (the paper's zero-block skipping): after the projector P_s of a crossing
    // gate on qubit t, and until the next non-diagonal gate on t, every amplitude whose bit t
    // differs from the path bit s is zero.  Pass plans keep the program order of the operations
    // on each qubit, so the set at the start of a pass follows from the program order of what
    // ran before it.
    std::vector<std::pair<uint8_t, uint8_t>> zs;
    auto zupdate = [&zs](const HalfOp &op) {
        if (op.kind == HK_PROJ) {
            const std::pair<uint8_t, uint8_t> e{op.q0, op.bit};
            if (std::find(zs.begin(), zs.end(), e) == zs.end()) zs.push_back(e);
        } else if (!is_diag(op.kind)) {
            const bool two = op.kind == HK_ISWAP;
            zs.erase(std::remove_if(zs.begin(), zs.end(),
                                    [&op, two](const std::pair<uint8_t, uint8_t> &e) {
                                        return e.first == op.q0 || (two && e.first == op.q1);
                                    }),
                     zs.end());
        }
    };
    // (with a prefix the parent state lacks the prefix's operations: start with no known zeros)
    if (!prefix)
        for (int l = 0; l < level0; ++l)
            for (const HalfOp &op : hp.segments[l]) zupdate(op);

    bool first = true;
    const bool dense_ok = dense_m >= 2 && n_ext >= 9 && q >= 4;
    while (first || !rem.empty()) {
        // a dense block on matrix cores (never the first pass of a segment, which reads the
        // parent batch or writes the initial state)
        if (!first && dense_ok) {
            std::vector<int> Q;
            std::vector<HalfOp> blk, dfr;
            uint64_t blocked = 0;
            int nd = 0;
            for (const HalfOp &op : rem) {
                const uint64_t qm = (uint64_t(1) << op.q0) | (is_two_qubit(op.kind) ? uint64_t(1) << op.q1 : 0);
                bool take = !(qm & blocked) && !is_branch(op.kind);
                std::vector<int> nq = Q;
                if (take) {
                    const int qq[2] = {op.q0, is_two_qubit(op.kind) ? (int)op.q1 : -1};
                    for (int x : qq) {
                        if (x < 0) continue;
                        if (p + x < 5) take = false;
                        if (std::find(nq.begin(), nq.end(), x) == nq.end()) nq.push_back(x);
                    }
                    if ((int)nq.size() > dense_m) take = false;
                }
                if (take) {
                    Q = nq;
                    blk.push_back(op);
                    if (!is_diag(op.kind)) ++nd;
                } else {
                    dfr.push_back(op);
                    blocked |= qm;
                }
            }
            if (nd >= 2) {
                for (int t = q - 1; t >= 0 && Q.size() < 4; --t)
                    if (p + t >= 5 && std::find(Q.begin(), Q.end(), t) == Q.end()) Q.push_back(t);
                std::sort(Q.begin(), Q.end());
                PassPlan pp;
                pp.dense = true;
                int qs[4];
                for (int t = 0; t < 4; ++t) { qs[t] = Q[t]; pp.bpos[t] = p + Q[t]; }
                pp.mat = dense_matrix(blk, qs);
                pp.n_nondiag = nd;
                for (const HalfOp &op : blk) carry += has_gain(op.kind) ? 1 : 0;   // norm gain sqrt2 each
                if (carry >= 32) {
                    const int e = std::min(carry / 2, seg_exp - taken);
                    pp.rescale_exp = e;
                    taken += e;
                    carry -= 2 * e;
                }
                pp.zero_in = zs;
                for (const HalfOp &op : blk) zupdate(op);
                pp.src = blk;
                sp.passes.push_back(std::move(pp));
                rem.swap(dfr);
                continue;
            }
        }
        first = false;
        PassPlan pp;
        std::vector<int> regq;
        std::vector<HalfOp> sched, defer;
        uint64_t blocked = 0;
        // lane bit 5 (and 4) may hold a chosen qubit (PassArgs::lane_qpos): when the slots fill all
        // six lane bits, where a qubit needs it; with fewer slot bits, always (a qubit without
        // gates in the pass fills it otherwise)
        int lq = -1, lq4 = -1;
        const bool lq_ok = max_lq >= 1 && (lq_small || (n_lane_q == 0 && p >= 6)) && q > R_eff;
        const bool lq4_ok = lq_ok && max_lq >= 2 && q > R_eff + 1;
        for (const HalfOp &op : rem) {
            const uint64_t qm = (uint64_t(1) << op.q0) | (is_two_qubit(op.kind) ? uint64_t(1) << op.q1 : 0);
            if (qm & blocked) { defer.push_back(op); blocked |= qm; continue; }
            if (!is_diag(op.kind)) {
                // every qubit of a non-diagonal op must sit in a lane bit or a register of this pass;
                // a qubit not yet placed takes a free register, else lane bit 5, else lane bit 4
                const int qs[2] = {op.q0, op.kind == HK_ISWAP ? (int)op.q1 : -1};
                std::vector<int> r2 = regq;
                int lq2 = lq, lq42 = lq4;
                bool fits = true;
                for (int t : qs) {
                    if (t < 0) continue;
                    const bool lane = t < n_lane_q || t == lq2 || t == lq42;
                    if (lane || std::find(r2.begin(), r2.end(), t) != r2.end()) continue;
                    if ((int)r2.size() < R_eff) r2.push_back(t);
                    else if (lq_ok && lq2 < 0) lq2 = t;
                    else if (lq4_ok && lq42 < 0) lq42 = t;
                    else fits = false;
                }
                if (fits) {
                    regq = r2;
                    lq = lq2;
                    lq4 = lq42;
                    sched.push_back(op);
                    continue;
                }
                defer.push_back(op);
                blocked |= qm;
                continue;
            }
            sched.push_back(op);
        }
        if (sched.empty() && !rem.empty()) {
            // only possible with no register bits while some qubit is outside the lane bits
            sp.ok = false;
            break;
        }
        // pad the register bits with untouched qubits so every tile holds 64 * 2^R_eff amplitudes
        for (int t = q - 1; t >= n_lane_q && (int)regq.size() < R_eff; --t)
            if (t != lq && t != lq4 && std::find(regq.begin(), regq.end(), t) == regq.end()) regq.push_back(t);
        if (lq_small) {
            // the freed lane bits must hold some qubit: the lowest one not placed yet
            auto free_q = [&]() {
                for (int t = n_lane_q; t < q; ++t)
                    if (t != lq && t != lq4 && std::find(regq.begin(), regq.end(), t) == regq.end()) return t;
                return -1;
            };
            if (lq < 0) lq = free_q();
            if (max_lq >= 2 && lq4 < 0) lq4 = free_q();
            if (lq < 0 || (max_lq >= 2 && lq4 < 0)) { sp.ok = false; break; }
        }
        std::sort(regq.begin(), regq.end());
        pp.R = (int)regq.size();
        pp.lane_q = lq;
        pp.lane_q4 = lq4;
        int kidx[64];
        for (int i = 0; i < 64; ++i) kidx[i] = -1;
        for (int k = 0; k < pp.R; ++k) {
            pp.reg_pos[k] = p + regq[k];
            kidx[p + regq[k]] = k;
        }
        PendingDiag pd;
        // position of a placed qubit: its lane bit, or its register index
        auto qpos = [&](int t, bool &lane) -> uint8_t {
            lane = t < n_lane_q || t == lq || t == lq4;
            return t == lq ? (uint8_t)5 : t == lq4 ? (uint8_t)4 : lane ? (uint8_t)(p + t) : (uint8_t)kidx[p + t];
        };
        for (const HalfOp &op : sched) {
            if (!is_diag(op.kind)) {
                const uint64_t qm = (uint64_t(1) << op.q0) | (op.kind == HK_ISWAP ? uint64_t(1) << op.q1 : 0);
                if (pd.touched & qm) flush(pd, pp, kidx);
                PassOp po;
                bool lane = false;
                po.target = qpos(op.q0, lane);
                po.pad = 0;
                if (op.kind == HK_ISWAP) {
                    bool lane1 = false;
                    po.type = PO_ISWAP;
                    po.group = qpos(op.q1, lane1);
                    po.kind = (uint8_t)((lane ? 1 : 0) | (lane1 ? 2 : 0));
                    pp.has_flip = true;          // the kernel variant that carries the two-qubit ops
                    ++pp.n_nondiag;
                    pp.ops.push_back(po);
                    continue;
                }
                if (op.kind == HK_PFLIP || op.kind == HK_PFLIPI) {
                    po.type = lane ? PO_PFLIP_LANE : PO_PFLIP_REG;
                    po.kind = op.kind == HK_PFLIPI ? 1 : 0;
                    po.group = op.bit;
                    pp.needs_slot_path = true;
                    pp.has_flip = true;
                } else {
                    po.type = lane ? PO_LANE : PO_REG;
                    po.kind = op.kind == HK_H ? GK_H : (op.kind == HK_X ? GK_X : GK_Y);
                    po.group = 0;
                    ++pp.n_nondiag;
                }
                pp.ops.push_back(po);
                continue;
            }
            switch (op.kind) {
            case HK_T:
                pd.lin[p + op.q0] = (pd.lin[p + op.q0] + 1) & 7;
                pd.touched |= uint64_t(1) << op.q0;
                break;
            case HK_CZ: {
                int a = p + op.q0, b = p + op.q1;
                if (a > b) std::swap(a, b);
                toggle(pd.quad, {a, b});
                pd.touched |= (uint64_t(1) << op.q0) | (uint64_t(1) << op.q1);
                break;
            }
            case HK_PROJ: {
                std::pair<int, int> e{p + op.q0, op.bit};
                if (std::find(pd.proj.begin(), pd.proj.end(), e) == pd.proj.end()) pd.proj.push_back(e);
                pd.touched |= uint64_t(1) << op.q0;
                break;
            }
            case HK_ZCTL:
                toggle(pd.zs, {p + op.q0, op.bit});
                pd.touched |= uint64_t(1) << op.q0;
                break;
            default:
                break;
            }
        }
        flush(pd, pp, kidx);
        // rescale: intermediate passes only when the gain got large, the last pass settles the segment
        for (const HalfOp &op : sched) carry += has_gain(op.kind) ? 1 : 0;
        if (carry >= 32) {
            const int e = std::min(carry / 2, seg_exp - taken);
            pp.rescale_exp = e;
            taken += e;
            carry -= 2 * e;
        }
        pp.zero_in = zs;
        for (const HalfOp &op : sched) zupdate(op);
        pp.src = sched;
        sp.passes.push_back(std::move(pp));
        rem.swap(defer);
    }
    sp.passes.back().rescale_exp += seg_exp - taken;
    return sp;
}

namespace {
// the plan with the fewest passes over lane-qubit choices: a qubit in a lane bit splits the
// contiguous runs of a load (two of 32 amplitudes, or four of 16 = one cache line each with
// two), so one or two are used only where that saves a pass
SegmentPlan best_plan(const Circuit &c, int half, int first, int last, int p, int R, int dense_m,
                      const std::vector<HalfOp> *prefix, int prefix_exp)
{
    SegmentPlan sp = plan_segment(c, half, first, last, p, R, dense_m, 0, prefix, prefix_exp);
    const int q = c.half[half].q;
    if (p >= 6 || q > 6 - p)
        for (int m = 1; m <= 2 && (p >= 6 || 6 - p - m >= 0); ++m) {
            SegmentPlan lq = plan_segment(c, half, first, last, p, R, dense_m, m, prefix, prefix_exp);
            if (lq.ok && (!sp.ok || lq.passes.size() < sp.passes.size())) sp = std::move(lq);
        }
    return sp;
}
}  // namespace

const SegmentPlan &get_segment_plan_range(Circuit &c, int half, int first, int last, int p, int R, int dense_m)
{
    const auto key = std::make_tuple(half, first, last, p, R, dense_m, -1, 0, 0);
    auto it = c.plan_cache.find(key);
    if (it != c.plan_cache.end()) return it->second;
    auto res = c.plan_cache.emplace(key, best_plan(c, half, first, last, p, R, dense_m, nullptr, 0));
    return res.first->second;
}

const SegmentPlan &get_segment_plan_tail(Circuit &c, int half, int first, int last, int p, int R, int dense_m,
                                         int pre_first, int pre_last, int pre_p)
{
    const auto key = std::make_tuple(half, first, last, p, R, dense_m, pre_first, pre_last, pre_p);
    auto it = c.plan_cache.find(key);
    if (it != c.plan_cache.end()) return it->second;
    const SegmentPlan &par = get_segment_plan_range(c, half, pre_first, pre_last, pre_p, R, dense_m);
    SegmentPlan sp;
    if (!par.ok || par.passes.size() < 2 || par.passes.back().dense) {
        sp.ok = false;
    } else {
        const std::vector<HalfOp> prefix = par.passes.back().src;
        sp = best_plan(c, half, first, last, p, R, dense_m, &prefix, par.passes.back().rescale_exp);
    }
    auto res = c.plan_cache.emplace(key, std::move(sp));
    return res.first->second;
}

const SegmentPlan &get_segment_plan(Circuit &c, int half, int level, int p, int R, int dense_m)
{
    return get_segment_plan_range(c, half, level, level, p, R, dense_m);
}

}  // namespace sf
