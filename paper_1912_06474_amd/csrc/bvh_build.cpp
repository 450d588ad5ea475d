// Host builder of the subdomain grid (the paper's sub-domains, Sec. 5) and
// of one binned-SAH BVH per subdomain.
//
// Grid: the bounding box of every triangle (light included), enlarged by
// 1e-3 of its largest extent so offset ray origins stay inside, split into
// nx * ny * nz equal cells.  The float planes are the single definition of
// the cells for every kernel.
//
// References: triangle i is referenced in every cell whose closed box
// overlaps its bounding box padded by 1e-4 of the scene extent (far above
// the FP32 position error of a hit point), so a hit whose parameter lies in
// a cell's interval is always found in that cell.  Each reference's box is
// the triangle box clipped to the padded cell.
//
// BVH: binned SAH over reference centroids, at most leaf_max references per
// leaf, depth capped at kMaxBvhDepth (a node at the cap becomes a leaf) so the
// traversal stack never overflows.  Child boxes are padded by 2e-6 of the
// scene extent so FP32 slab tests cannot reject a box that holds a hit.
//
// Node storage: each child box is quantised to 16 bits per coordinate on a
// per-cell lattice base + q * step spanning the cell's root box, rounded
// outward so the FP32 lattice value fmaf(q, step, base) never cuts into the
// padded box.  A node is two 16-byte children (boxes + link): half the bytes
// of float boxes, with the same traversal result (a looser box only costs
// visits; every triangle is still tested exactly).
#include "bvh_build.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "layout.h"

namespace sdd {

namespace {

struct Ref {
    float lo[3], hi[3];
    float c[3];
    int prim;
};

struct BNode {
    float lo[3], hi[3];
    int left = -1, right = -1;  // children (BNode indices) or -1 for a leaf
    int first = 0, count = 0;   // leaf range in the cell's ref array
    int depth = 0;
};

float round_down(double v) {
    float f = (float)v;
    if ((double)f > v) f = std::nextafter(f, -INFINITY);
    return f;
}
float round_up(double v) {
    float f = (float)v;
    if ((double)f < v) f = std::nextafter(f, INFINITY);
    return f;
}

// per-cell lattice: fmaf(q, step, base) for q in [0, 65535] covers [lo, hi]
void lattice(float lo, float hi, float& base, float& step) {
    base = lo;
    if (!(hi > lo)) {
        step = 0.0f;
        return;
    }
    step = round_up(((double)hi - (double)lo) / 65535.0);
    while (std::fmaf(65535.0f, step, base) < hi) step = std::nextafter(step, INFINITY);
}

// outward-rounded lattice coordinates of [lo, hi] (clamped to the lattice)
uint32_t quant_lo(float v, float base, float step) {
    if (!(step > 0.0f)) return 0;
    double q = std::floor(((double)v - (double)base) / (double)step);
    int qi = (int)std::min(65535.0, std::max(0.0, q));
    while (qi > 0 && std::fmaf((float)qi, step, base) > v) --qi;
    return (uint32_t)qi;
}
uint32_t quant_hi(float v, float base, float step) {
    if (!(step > 0.0f)) return 0;
    double q = std::ceil(((double)v - (double)base) / (double)step);
    int qi = (int)std::min(65535.0, std::max(0.0, q));
    while (qi < 65535 && std::fmaf((float)qi, step, base) < v) ++qi;
    return (uint32_t)qi;
}

float half_area(const float lo[3], const float hi[3]) {
    const float dx = std::max(0.0f, hi[0] - lo[0]), dy = std::max(0.0f, hi[1] - lo[1]),
                dz = std::max(0.0f, hi[2] - lo[2]);
    return dx * dy + dy * dz + dz * dx;
}

struct CellBuilder {
    std::vector<Ref> refs;
    std::vector<BNode> nodes;
    int leaf_max = 4;
    int bins = 16;
    int max_depth = 0;

    int build(int first, int count, int depth) {
        BNode nd;
        nd.depth = depth;
        max_depth = std::max(max_depth, depth);
        float clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int a = 0; a < 3; ++a) {
            nd.lo[a] = INFINITY;
            nd.hi[a] = -INFINITY;
        }
        for (int i = first; i < first + count; ++i) {
            const Ref& r = refs[i];
            for (int a = 0; a < 3; ++a) {
                nd.lo[a] = std::min(nd.lo[a], r.lo[a]);
                nd.hi[a] = std::max(nd.hi[a], r.hi[a]);
                clo[a] = std::min(clo[a], r.c[a]);
                chi[a] = std::max(chi[a], r.c[a]);
            }
        }
        const int id = (int)nodes.size();
        nodes.push_back(nd);
        if (count <= leaf_max || depth + 1 >= kMaxBvhDepth) {
            nodes[id].first = first;
            nodes[id].count = count;
            return id;
        }
        // binned SAH
        int best_axis = -1, best_bin = -1;
        float best_cost = INFINITY;
        std::vector<int> cnt(bins);
        std::vector<float> blo(bins * 3), bhi(bins * 3);
        std::vector<float> lcost(bins);
        for (int a = 0; a < 3; ++a) {
            const float ext = chi[a] - clo[a];
            if (!(ext > 0.0f)) continue;
            const float scale = (float)bins / ext;
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int b = 0; b < bins; ++b)
                for (int k = 0; k < 3; ++k) {
                    blo[3 * b + k] = INFINITY;
                    bhi[3 * b + k] = -INFINITY;
                }
            for (int i = first; i < first + count; ++i) {
                const Ref& r = refs[i];
                int b = (int)((r.c[a] - clo[a]) * scale);
                b = std::min(std::max(b, 0), bins - 1);
                ++cnt[b];
                for (int k = 0; k < 3; ++k) {
                    blo[3 * b + k] = std::min(blo[3 * b + k], r.lo[k]);
                    bhi[3 * b + k] = std::max(bhi[3 * b + k], r.hi[k]);
                }
            }
            float alo[3] = {INFINITY, INFINITY, INFINITY}, ahi[3] = {-INFINITY, -INFINITY, -INFINITY};
            int n_left = 0;
            for (int b = 0; b < bins - 1; ++b) {
                n_left += cnt[b];
                for (int k = 0; k < 3; ++k) {
                    alo[k] = std::min(alo[k], blo[3 * b + k]);
                    ahi[k] = std::max(ahi[k], bhi[3 * b + k]);
                }
                lcost[b] = n_left ? half_area(alo, ahi) * (float)n_left : INFINITY;
                if (!n_left) lcost[b] = -1.0f;
            }
            float rlo[3] = {INFINITY, INFINITY, INFINITY}, rhi[3] = {-INFINITY, -INFINITY, -INFINITY};
            int n_right = 0;
            for (int b = bins - 1; b >= 1; --b) {
                n_right += cnt[b];
                for (int k = 0; k < 3; ++k) {
                    rlo[k] = std::min(rlo[k], blo[3 * b + k]);
                    rhi[k] = std::max(rhi[k], bhi[3 * b + k]);
                }
                const int split = b - 1;  // left = bins [0, split]
                const int nl = count - n_right;
                if (nl <= 0 || n_right <= 0 || lcost[split] < 0.0f) continue;
                const float cost = lcost[split] + half_area(rlo, rhi) * (float)n_right;
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_bin = split;
                }
            }
        }
        int mid;
        if (best_axis < 0) {
            mid = first + count / 2;  // all centroids coincide: any halving is as good
        } else {
            const float ext = chi[best_axis] - clo[best_axis];
            const float scale = (float)bins / ext;
            const float c0 = clo[best_axis];
            const int a = best_axis, split = best_bin, nb = bins;
            auto it = std::partition(refs.begin() + first, refs.begin() + first + count, [&](const Ref& r) {
                int b = (int)((r.c[a] - c0) * scale);
                b = std::min(std::max(b, 0), nb - 1);
                return b <= split;
            });
            mid = (int)(it - refs.begin());
            if (mid == first || mid == first + count) mid = first + count / 2;
        }
        const int l = build(first, mid - first, depth + 1);
        const int r = build(mid, first + count - mid, depth + 1);
        nodes[id].left = l;
        nodes[id].right = r;
        return id;
    }
};

}  // namespace

void triangle_info(const BuildInput& in, std::vector<HostF4>& info) {
    info.resize(in.n_tris);
    for (int i = 0; i < in.n_tris; ++i) {
        const int32_t* t = in.tris + 3 * (size_t)i;
        double v[3][3];
        for (int j = 0; j < 3; ++j)
            for (int a = 0; a < 3; ++a) v[j][a] = (double)in.verts[3 * (size_t)t[j] + a];
        const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
        const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
        const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                             e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        const double s = len > 0.0 ? 1.0 / len : 0.0;
        const int32_t mat = in.tri_mat[i];
        const int32_t typ = in.mat_type[mat] & 3;
        const int32_t id = (typ == kGlass && in.glass_of) ? in.glass_of[mat] : mat;
        const int32_t word = id | (typ << kMatTypeShift) | ((in.mat_emits && in.mat_emits[mat]) ? kMatEmits : 0);
        float w;
        std::memcpy(&w, &word, 4);
        info[i] = HostF4{(float)(n[0] * s), (float)(n[1] * s), (float)(n[2] * s), w};
    }
}

bool grid_planes(const BuildInput& in, GridBvh& out, double& ext, std::string& err) {
    const int T = in.n_tris;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = 0; i < T; ++i)
        for (int j = 0; j < 3; ++j) {
            const float* p = in.verts + 3 * (size_t)in.tris[3 * (size_t)i + j];
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], (double)p[a]);
                hi[a] = std::max(hi[a], (double)p[a]);
            }
        }
    ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, hi[a] - lo[a]);
    if (!(ext > 0.0) || !std::isfinite(ext)) {
        err = "scene has no spatial extent";
        return false;
    }
    const double gpad = 1e-3 * ext;
    const int n[3] = {in.nx, in.ny, in.nz};
    out.nx = in.nx;
    out.ny = in.ny;
    out.nz = in.nz;
    out.planes.clear();
    for (int a = 0; a < 3; ++a) {
        const double g0 = lo[a] - gpad, g1 = hi[a] + gpad;
        out.lo[a] = g0;
        out.hi[a] = g1;
        std::vector<float> pl(n[a] + 1);
        for (int i = 0; i <= n[a]; ++i) pl[i] = (float)(g0 + (g1 - g0) * (double)i / (double)n[a]);
        pl[0] = round_down(g0);
        pl[n[a]] = round_up(g1);
        for (int i = 0; i < n[a]; ++i)
            if (!(pl[i + 1] > pl[i])) {
                err = "subdomain grid too fine for FP32 planes";
                return false;
            }
        out.planes.insert(out.planes.end(), pl.begin(), pl.end());
    }
    return true;
}

bool build_grid_bvh(const BuildInput& in, GridBvh& out, std::string& err) {
    const int T = in.n_tris;
    double ext = 0.0;
    if (!grid_planes(in, out, ext, err)) return false;
    const double cpad = 1e-4 * ext, npad = 2e-6 * ext;
    const int n[3] = {in.nx, in.ny, in.nz};
    std::vector<float> pl[3];
    for (int a = 0, o = 0; a < 3; o += n[a] + 1, ++a) pl[a].assign(out.planes.begin() + o, out.planes.begin() + o + n[a] + 1);
    const int G = n[0] * n[1] * n[2];

    // references per cell
    std::vector<std::vector<Ref>> cell_refs(G);
    for (int i = 0; i < T; ++i) {
        double tlo[3] = {INFINITY, INFINITY, INFINITY}, thi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int j = 0; j < 3; ++j) {
            const float* p = in.verts + 3 * (size_t)in.tris[3 * (size_t)i + j];
            for (int a = 0; a < 3; ++a) {
                tlo[a] = std::min(tlo[a], (double)p[a]);
                thi[a] = std::max(thi[a], (double)p[a]);
            }
        }
        int r0[3], r1[3];
        for (int a = 0; a < 3; ++a) {
            const double plo = tlo[a] - cpad, phi = thi[a] + cpad;
            int i0 = 0;
            while (i0 < n[a] - 1 && (double)pl[a][i0 + 1] < plo) ++i0;
            int i1 = n[a] - 1;
            while (i1 > 0 && (double)pl[a][i1] > phi) --i1;
            r0[a] = i0;
            r1[a] = i1;
        }
        for (int iz = r0[2]; iz <= r1[2]; ++iz)
            for (int iy = r0[1]; iy <= r1[1]; ++iy)
                for (int ix = r0[0]; ix <= r1[0]; ++ix) {
                    const int ci[3] = {ix, iy, iz};
                    Ref r;
                    for (int a = 0; a < 3; ++a) {
                        const double clo = (double)pl[a][ci[a]] - cpad, chi = (double)pl[a][ci[a] + 1] + cpad;
                        r.lo[a] = round_down(std::max(tlo[a], clo) - npad);
                        r.hi[a] = round_up(std::min(thi[a], chi) + npad);
                        r.c[a] = 0.5f * (r.lo[a] + r.hi[a]);
                    }
                    r.prim = i;
                    cell_refs[ix + n[0] * (iy + n[1] * iz)].push_back(r);
                }
    }

    // per-cell BVHs, in parallel
    std::vector<CellBuilder> cb(G);
    std::atomic<int> next{0};
    const int nthreads = std::max(1, std::min<int>(G, (int)std::thread::hardware_concurrency()));
    auto work = [&]() {
        for (;;) {
            const int c = next.fetch_add(1);
            if (c >= G) break;
            CellBuilder& b = cb[c];
            b.refs.swap(cell_refs[c]);
            b.leaf_max = in.leaf_max;
            b.bins = in.sah_bins;
            b.nodes.reserve(2 * b.refs.size() / std::max(1, in.leaf_max) + 2);
            if (!b.refs.empty()) b.build(0, (int)b.refs.size(), 0);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nthreads; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();

    // flatten: breadth-first inner nodes; leaves become links to triangle runs
    out.nodes.clear();
    out.tris.clear();
    out.cell_q.assign(2 * (size_t)G, HostF4{0.0f, 0.0f, 0.0f, 0.0f});
    out.cell_root.assign(G, 0);
    out.cell_refs.assign(G, 0);
    out.cell_nodes.assign(G, 0);
    out.n_refs = 0;
    out.max_depth = 0;
    const float far = 1e30f;
    auto int_bits = [](int v) {
        float f;
        std::memcpy(&f, &v, 4);
        return f;
    };
    for (int c = 0; c < G; ++c) {
        CellBuilder& b = cb[c];
        out.max_depth = std::max(out.max_depth, b.max_depth);
        out.cell_refs[c] = (int)b.refs.size();
        out.n_refs += (int64_t)b.refs.size();
        const int node_base = (int)(out.nodes.size() / 8);
        // inner nodes in BFS order; a root leaf (or an empty cell) gets a wrapper
        std::vector<int> bfs;
        std::vector<int> gid(b.nodes.size(), -1);
        const bool wrap = b.nodes.empty() || b.nodes[0].left < 0;
        if (!wrap) {
            bfs.push_back(0);
            gid[0] = 0;
            for (size_t k = 0; k < bfs.size(); ++k) {
                const BNode& nd = b.nodes[bfs[k]];
                for (int ch : {nd.left, nd.right})
                    if (b.nodes[ch].left >= 0) {
                        gid[ch] = (int)bfs.size();
                        bfs.push_back(ch);
                    }
            }
        }
        const int n_inner = wrap ? 1 : (int)bfs.size();
        out.cell_root[c] = node_base;
        out.cell_nodes[c] = n_inner;
        out.nodes.resize(out.nodes.size() + 8 * (size_t)n_inner);
        // lattice over the cell's root box (the union of its references)
        float qbase[3] = {0.0f, 0.0f, 0.0f}, qstep[3] = {0.0f, 0.0f, 0.0f};
        if (!b.refs.empty())
            for (int a = 0; a < 3; ++a) lattice(b.nodes[0].lo[a], b.nodes[0].hi[a], qbase[a], qstep[a]);
        out.cell_q[2 * (size_t)c] = HostF4{qbase[0], qbase[1], qbase[2], 0.0f};
        out.cell_q[2 * (size_t)c + 1] = HostF4{qstep[0], qstep[1], qstep[2], 0.0f};
        auto emit_leaf = [&](const BNode& lf) {
            const int start = (int)(out.tris.size() / 3);
            for (int i = lf.first; i < lf.first + lf.count; ++i) {
                const int prim = b.refs[i].prim;
                const int32_t* t = in.tris + 3 * (size_t)prim;
                const float* v0 = in.verts + 3 * (size_t)t[0];
                const float* v1 = in.verts + 3 * (size_t)t[1];
                const float* v2 = in.verts + 3 * (size_t)t[2];
                const int mat = in.tri_mat[prim];
                const int meta = (in.mat_type[mat] & 3) | (i == lf.first + lf.count - 1 ? kLastInLeaf : 0);
                const int gi = in.glass_of ? in.glass_of[mat] : -1;
                out.tris.push_back(HostF4{v0[0], v0[1], v0[2], int_bits(prim)});
                out.tris.push_back(HostF4{(float)((double)v1[0] - v0[0]), (float)((double)v1[1] - v0[1]),
                                          (float)((double)v1[2] - v0[2]), int_bits(meta)});
                out.tris.push_back(HostF4{(float)((double)v2[0] - v0[0]), (float)((double)v2[1] - v0[1]),
                                          (float)((double)v2[2] - v0[2]), int_bits(gi)});
            }
            return ~start;
        };
        auto child = [&](int ch, float blo[3], float bhi[3]) -> int {
            if (ch < 0) {
                for (int a = 0; a < 3; ++a) blo[a] = bhi[a] = far;
                return kEmptyLink;
            }
            const BNode& nd = b.nodes[ch];
            for (int a = 0; a < 3; ++a) {
                blo[a] = nd.lo[a];
                bhi[a] = nd.hi[a];
            }
            if (nd.left < 0) return nd.count > 0 ? emit_leaf(nd) : kEmptyLink;
            return node_base + gid[ch];
        };
        for (int k = 0; k < n_inner; ++k) {
            int ch0 = -1, ch1 = -1;
            if (wrap) {
                ch0 = b.nodes.empty() ? -1 : 0;
            } else {
                ch0 = b.nodes[bfs[k]].left;
                ch1 = b.nodes[bfs[k]].right;
            }
            float lo0[3], hi0[3], lo1[3], hi1[3];
            const int l0 = child(ch0, lo0, hi0);
            const int l1 = child(ch1, lo1, hi1);
            uint32_t* nd = &out.nodes[8 * (size_t)(node_base + k)];
            const float* clo[2] = {lo0, lo1};
            const float* chi[2] = {hi0, hi1};
            const int lk[2] = {l0, l1};
            for (int i = 0; i < 2; ++i) {
                for (int a = 0; a < 3; ++a) {
                    uint32_t ql = 0, qh = 0;
                    if (lk[i] != kEmptyLink) {
                        ql = quant_lo(clo[i][a], qbase[a], qstep[a]);
                        qh = quant_hi(chi[i][a], qbase[a], qstep[a]);
                    }
                    nd[4 * i + a] = ql | (qh << 16);
                }
                nd[4 * i + 3] = (uint32_t)lk[i];
            }
        }
    }
    return true;
}

}  // namespace sdd
