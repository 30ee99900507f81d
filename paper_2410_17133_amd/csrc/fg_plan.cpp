// Host planning of a mesh: node graph, row permutation, sliced block-ELL
// layout, tetrahedron colouring and interface adjacency.  Runs once per mesh.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "fg_internal.h"

namespace fg {

namespace {

int n_threads()
{
    unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 16u));
}

template <class F>
void parallel_for(int64_t n, F f)
{
    int T = n_threads();
    if (n < 4096 || T == 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + T - 1) / T;
    for (int t = 0; t < T; ++t) {
        int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a < b) th.emplace_back([=] { f(a, b); });
    }
    for (auto &x : th) x.join();
}

// Interleave the low 21 bits of v with two zero bits between each.
uint64_t spread3(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

}  // namespace

fg_status build_plan(const fg_mesh &m, Plan &P, std::string &err)
{
    const int64_t N = m.n_nodes, ne = m.n_tets, nf = m.n_coh;
    if (N <= 0 || ne <= 0 || !m.xyz_h || !m.tets_h || !m.dir_u_h || !m.dir_p_h || (nf > 0 && !m.coh_h)) {
        err = "fg_system_create: empty mesh or null array";
        return FG_ERR_ARG;
    }
    if (N >= (int64_t)INT32_MAX || ne >= (int64_t)INT32_MAX / 4) {
        err = "fg_system_create: mesh too large for 32-bit indices";
        return FG_ERR_ARG;
    }
    for (int64_t i = 0; i < ne * 4; ++i)
        if (m.tets_h[i] < 0 || m.tets_h[i] >= N) {
            err = "fg_system_create: tetrahedron node id out of range";
            return FG_ERR_ARG;
        }
    for (int64_t i = 0; i < nf * 6; ++i)
        if (m.coh_h[i] < 0 || m.coh_h[i] >= N) {
            err = "fg_system_create: interface node id out of range";
            return FG_ERR_ARG;
        }
    P.N = N;
    P.ne = ne;
    P.nf = nf;

    // node -> incident element lists (tets first, then interface elements as ne + t)
    std::vector<int64_t> inc_ptr(N + 1, 0);
    for (int64_t i = 0; i < ne * 4; ++i) inc_ptr[m.tets_h[i] + 1]++;
    for (int64_t i = 0; i < nf * 6; ++i) inc_ptr[m.coh_h[i] + 1]++;
    for (int64_t i = 0; i < N; ++i) inc_ptr[i + 1] += inc_ptr[i];
    std::vector<int64_t> inc(inc_ptr[N]);
    {
        std::vector<int64_t> pos(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e)
            for (int a = 0; a < 4; ++a) inc[pos[m.tets_h[4 * e + a]]++] = e;
        for (int64_t t = 0; t < nf; ++t)
            for (int a = 0; a < 6; ++a) inc[pos[m.coh_h[6 * t + a]]++] = ne + t;
    }
    // neighbour sets (caller ids, ascending) with row lengths
    std::vector<int32_t> rlen(N);
    parallel_for(N, [&](int64_t a, int64_t b) {
        std::vector<int32_t> buf;
        for (int64_t i = a; i < b; ++i) {
            buf.clear();
            for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
                int64_t e = inc[k];
                if (e < ne)
                    for (int v = 0; v < 4; ++v) buf.push_back(m.tets_h[4 * e + v]);
                else
                    for (int v = 0; v < 6; ++v) buf.push_back(m.coh_h[6 * (e - ne) + v]);
            }
            std::sort(buf.begin(), buf.end());
            rlen[i] = (int32_t)(std::unique(buf.begin(), buf.end()) - buf.begin());
        }
    });
    int maxlen = *std::max_element(rlen.begin(), rlen.end());
    if (maxlen > 255) {
        err = "fg_system_create: a node has more than 255 graph neighbours";
        return FG_ERR_ARG;
    }

    // Row order: longest rows first (so slices hold rows of equal length and
    // need almost no padding), then a Morton order of the coordinates so that
    // the x-gathers of a slice and of neighbouring slices hit the same lines.
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < N; ++i)
        for (int r = 0; r < 3; ++r) {
            lo[r] = std::min(lo[r], m.xyz_h[3 * i + r]);
            hi[r] = std::max(hi[r], m.xyz_h[3 * i + r]);
        }
    double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    std::vector<uint64_t> code(N);
    for (int64_t i = 0; i < N; ++i) {
        uint64_t c = 0;
        for (int r = 0; r < 3; ++r) {
            double f = (m.xyz_h[3 * i + r] - lo[r]) / ext;
            uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, f * 2097151.0));
            c |= spread3(q) << r;
        }
        code[i] = c;
    }
    // Groups (independent instances of a batch): rows of a group are contiguous
    // and each group is padded to whole slices, so a slice never mixes groups.
    std::vector<int32_t> grp(N, 0);
    int ngroups = 1;
    if (m.group_h) {
        int gmax = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (m.group_h[i] < 0 || m.group_h[i] >= MAX_GROUPS) {
                err = "fg_system_create: group id out of range [0, 64)";
                return FG_ERR_ARG;
            }
            grp[i] = m.group_h[i];
            gmax = std::max(gmax, (int)grp[i]);
        }
        ngroups = gmax + 1;
        // an element must not couple two groups
        for (int64_t e = 0; e < ne; ++e)
            for (int a = 1; a < 4; ++a)
                if (grp[m.tets_h[4 * e + a]] != grp[m.tets_h[4 * e]]) {
                    err = "fg_system_create: a tetrahedron spans two groups";
                    return FG_ERR_ARG;
                }
        for (int64_t t = 0; t < nf; ++t)
            for (int a = 1; a < 6; ++a)
                if (grp[m.coh_h[6 * t + a]] != grp[m.coh_h[6 * t]]) {
                    err = "fg_system_create: an interface element spans two groups";
                    return FG_ERR_ARG;
                }
    }
    std::vector<int32_t> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (grp[a] != grp[b]) return grp[a] < grp[b];
        if (rlen[a] != rlen[b]) return rlen[a] > rlen[b];
        if (code[a] != code[b]) return code[a] < code[b];
        return a < b;
    });
    P.ngroups = ngroups;
    P.group_slice_ptr.assign(ngroups + 1, 0);
    P.perm.clear();
    {
        int64_t k = 0;
        for (int g = 0; g < ngroups; ++g) {
            while (k < N && grp[order[k]] == g) P.perm.push_back(order[k++]);
            while (P.perm.size() % SLICE) P.perm.push_back(-1);  // padding rows close the group's last slice
            P.group_slice_ptr[g + 1] = (int64_t)P.perm.size() / SLICE;
        }
    }
    P.iperm.assign(N, 0);
    for (int64_t r = 0; r < (int64_t)P.perm.size(); ++r)
        if (P.perm[r] >= 0) P.iperm[P.perm[r]] = (int32_t)r;

    // sliced block-ELL layout
    P.Npad = (int64_t)P.perm.size();
    P.nslices = P.Npad / SLICE;
    P.slice_group.assign(P.nslices, 0);
    for (int g = 0; g < ngroups; ++g)
        for (int64_t s = P.group_slice_ptr[g]; s < P.group_slice_ptr[g + 1]; ++s) P.slice_group[s] = g;
    P.slice_ptr.assign(P.nslices + 1, 0);
    for (int64_t s = 0; s < P.nslices; ++s) {
        int w = 0;
        for (int l = 0; l < SLICE; ++l) {
            int64_t r = s * SLICE + l;
            if (P.perm[r] >= 0) w = std::max(w, (int)rlen[P.perm[r]]);
        }
        P.slice_ptr[s + 1] = P.slice_ptr[s] + (int64_t)w * SLICE;
    }
    P.nblk_pad = P.slice_ptr[P.nslices];
    P.col.assign(P.nblk_pad, 0);
    P.rowlen.assign(P.Npad, 0);
    P.diag_slot.assign(P.Npad, -1);
    std::atomic<int64_t> npairs{0};
    parallel_for(P.Npad, [&](int64_t a, int64_t b) {
        std::vector<int32_t> buf;
        int64_t local = 0;
        for (int64_t r = a; r < b; ++r) {
            int64_t s = r / SLICE, l = r % SLICE;
            int64_t base = P.slice_ptr[s];
            int w = (int)((P.slice_ptr[s + 1] - base) / SLICE);
            buf.clear();
            if (P.perm[r] >= 0) {
                int64_t i = P.perm[r];
                for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
                    int64_t e = inc[k];
                    if (e < ne)
                        for (int v = 0; v < 4; ++v) buf.push_back(P.iperm[m.tets_h[4 * e + v]]);
                    else
                        for (int v = 0; v < 6; ++v) buf.push_back(P.iperm[m.coh_h[6 * (e - ne) + v]]);
                }
                std::sort(buf.begin(), buf.end());
                buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
            }
            P.rowlen[r] = (uint8_t)buf.size();
            local += (int64_t)buf.size();
            for (int j = 0; j < w; ++j) {
                int32_t c = j < (int)buf.size() ? buf[j] : (int32_t)r;
                P.col[base + (int64_t)j * SLICE + l] = c;
                if (j < (int)buf.size() && c == r) P.diag_slot[r] = j;
            }
        }
        npairs += local;
    });
    P.npairs = npairs.load();

    // Per-slice halo: the sorted distinct columns of the slice's rows.  The
    // products stage x of the halo in LDS and address it with 16-bit local
    // column indices.
    P.halo_ptr.assign(P.nslices + 1, 0);
    std::vector<std::vector<int32_t>> halos(P.nslices);
    P.lcol.assign(P.nblk_pad, 0);
    parallel_for(P.nslices, [&](int64_t a, int64_t b) {
        for (int64_t s = a; s < b; ++s) {
            const int64_t base = P.slice_ptr[s];
            const int64_t len = P.slice_ptr[s + 1] - base;
            std::vector<int32_t> &h = halos[s];
            h.assign(P.col.begin() + base, P.col.begin() + base + len);
            std::sort(h.begin(), h.end());
            h.erase(std::unique(h.begin(), h.end()), h.end());
            for (int64_t k = 0; k < len; ++k)
                P.lcol[base + k] = (uint16_t)(std::lower_bound(h.begin(), h.end(), P.col[base + k]) - h.begin());
        }
    });
    for (int64_t s = 0; s < P.nslices; ++s) {
        P.halo_ptr[s + 1] = P.halo_ptr[s] + (int64_t)halos[s].size();
        P.halo_max = std::max<int64_t>(P.halo_max, (int64_t)halos[s].size());
    }
    P.halo.resize(P.halo_ptr[P.nslices]);
    for (int64_t s = 0; s < P.nslices; ++s) std::copy(halos[s].begin(), halos[s].end(), P.halo.begin() + P.halo_ptr[s]);

    // greedy colouring of tetrahedra: no two tetrahedra of a colour share a node
    const int MAXC = 256;
    std::vector<uint64_t> used((size_t)N * (MAXC / 64), 0);
    std::vector<int16_t> colour(ne);
    int ncol = 0;
    for (int64_t e = 0; e < ne; ++e) {
        uint64_t forb[MAXC / 64] = {0};
        for (int a = 0; a < 4; ++a) {
            const uint64_t *u = &used[(size_t)m.tets_h[4 * e + a] * (MAXC / 64)];
            for (int w = 0; w < MAXC / 64; ++w) forb[w] |= u[w];
        }
        int c = -1;
        for (int w = 0; w < MAXC / 64 && c < 0; ++w)
            if (~forb[w]) c = 64 * w + __builtin_ctzll(~forb[w]);
        if (c < 0) {
            err = "fg_system_create: more than 256 colours needed";
            return FG_ERR_ARG;
        }
        colour[e] = (int16_t)c;
        ncol = std::max(ncol, c + 1);
        for (int a = 0; a < 4; ++a) used[(size_t)m.tets_h[4 * e + a] * (MAXC / 64) + c / 64] |= 1ULL << (c % 64);
    }
    P.colour_ptr.assign(ncol + 1, 0);
    for (int64_t e = 0; e < ne; ++e) P.colour_ptr[colour[e] + 1]++;
    for (int c = 0; c < ncol; ++c) P.colour_ptr[c + 1] += P.colour_ptr[c];
    P.tets.resize(ne * 4);
    P.tet_orig.resize(ne);
    {
        std::vector<int64_t> pos(P.colour_ptr.begin(), P.colour_ptr.end() - 1);
        for (int64_t e = 0; e < ne; ++e) {
            int64_t k = pos[colour[e]]++;
            P.tet_orig[k] = (int32_t)e;
            for (int a = 0; a < 4; ++a) P.tets[4 * k + a] = P.iperm[m.tets_h[4 * e + a]];
        }
    }

    // interface elements: internal ids, fault rows and their incident elements
    P.coh.resize(nf * 6);
    for (int64_t i = 0; i < nf * 6; ++i) P.coh[i] = P.iperm[m.coh_h[i]];
    for (int64_t t = 0; t < nf; ++t) {
        const double *x = m.xyz_h;
        const int32_t *c = m.coh_h + 6 * t;
        double e1[3], e2[3];
        for (int r = 0; r < 3; ++r) {
            e1[r] = x[3 * c[4] + r] - x[3 * c[3] + r];
            e2[r] = x[3 * c[5] + r] - x[3 * c[3] + r];
        }
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        if (!(std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]) > 0)) {
            err = "fg_system_create: degenerate interface triangle";
            return FG_ERR_ARG;
        }
    }
    {
        std::vector<int32_t> is_f(P.Npad, -1);
        for (int64_t i = 0; i < nf * 6; ++i) is_f[P.coh[i]] = 0;
        for (int64_t r = 0; r < P.Npad; ++r)
            if (is_f[r] == 0) {
                is_f[r] = (int32_t)P.frows.size();
                P.frows.push_back((int32_t)r);
            }
        P.fadj_ptr.assign(P.frows.size() + 1, 0);
        for (int64_t i = 0; i < nf * 6; ++i) P.fadj_ptr[is_f[P.coh[i]] + 1]++;
        for (size_t k = 0; k < P.frows.size(); ++k) P.fadj_ptr[k + 1] += P.fadj_ptr[k];
        P.fadj.resize(P.fadj_ptr.back());
        std::vector<int32_t> pos(P.fadj_ptr.begin(), P.fadj_ptr.end() - 1);
        for (int64_t i = 0; i < nf * 6; ++i) P.fadj[pos[is_f[P.coh[i]]]++] = (int32_t)i;
        // the two lips' nodes at the same point pair up; a node met with two
        // different partners keeps none (its block stays 3x3)
        P.fslot = is_f;
        P.fpart.assign(P.frows.size(), -1);
        std::vector<uint8_t> bad(P.frows.size(), 0);
        for (int64_t t = 0; t < nf; ++t)
            for (int a = 0; a < 3; ++a) {
                const int32_t u = P.coh[6 * t + a], v = P.coh[6 * t + 3 + a];
                for (int side = 0; side < 2; ++side) {
                    const int32_t x = side ? v : u, y = side ? u : v;
                    const int32_t k = is_f[x];
                    if (P.fpart[k] >= 0 && P.fpart[k] != y) bad[k] = 1;
                    P.fpart[k] = y;
                }
            }
        for (size_t k = 0; k < P.frows.size(); ++k)
            if (bad[k] || P.fpart[k] == P.frows[k]) P.fpart[k] = -1;
        for (size_t k = 0; k < P.frows.size(); ++k)   // keep the map symmetric
            if (P.fpart[k] >= 0 && P.fpart[is_f[P.fpart[k]]] != P.frows[k]) P.fpart[k] = -1;
    }

    P.dir_u.assign(3 * P.Npad, 0);
    P.dir_p.assign(P.Npad, 0);
    for (int64_t r = 0; r < P.Npad; ++r) {
        const int64_t i = P.perm[r];
        if (i < 0) continue;
        for (int c = 0; c < 3; ++c) P.dir_u[3 * r + c] = m.dir_u_h[3 * i + c] ? 1 : 0;
        P.dir_p[r] = m.dir_p_h[i] ? 1 : 0;
    }
    return FG_OK;
}

}  // namespace fg
