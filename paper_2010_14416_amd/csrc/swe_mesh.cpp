// Host-side mesh preparation (once per mesh). See swe_mesh.hpp.
//
// Conventions shared with the interface (include/swe.h):
//  * a clockwise triangle is reoriented by exchanging its second and third
//    vertex; local side k of a triangle runs from vertex k to vertex k+1;
//  * the left cell of an interior edge is the one whose counter-clockwise
//    boundary traverses the edge from its lower to its higher node number,
//    and the edge normal points from the left to the right cell; on the
//    boundary the only cell is the left one and the normal points outward.
// Both are interface conventions: any implementation of the method on the
// same node numbering gets the same edge orientation, whatever the cell
// order.
#include "swe_mesh.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace swe {
namespace {

template <typename... A>
std::string fmt(const char *f, A... a)
{
    char buf[512];
    std::snprintf(buf, sizeof buf, f, a...);
    return buf;
}

// Index along a Hilbert curve of order 16 of the lattice point (x, y),
// 0 <= x, y < 2^16 (Hilbert 1891; the usual quadrant-rotation recurrence).
uint32_t hilbert_index(uint32_t x, uint32_t y)
{
    const uint32_t n = 1u << 16;
    uint32_t d = 0;
    for (uint32_t s = n >> 1; s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1u : 0u;
        uint32_t ry = (y & s) ? 1u : 0u;
        d += s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = n - 1 - x;
                y = n - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

}  // namespace

bool build_block_mesh(int64_t nn, const double *xy, int64_t nc,
                      const int32_t *tri_in, int64_t nbnd,
                      const int32_t *bnd_nodes, const int32_t *bnd_tag,
                      int32_t block_cells, bool reorder, int32_t max_tag,
                      BlockMesh &M, std::string &err)
{
    M = BlockMesh();
    if (nn < 3 || nc < 1) {
        err = "mesh needs at least 3 nodes and 1 triangle";
        return false;
    }
    if (nn > INT32_MAX || nc > INT32_MAX / 3) {
        err = "mesh too large for 32-bit indices";
        return false;
    }
    for (int64_t k = 0; k < 2 * nn; ++k)
        if (!std::isfinite(xy[k])) {
            err = fmt("node %lld has a non-finite coordinate",
                      (long long)(k / 2));
            return false;
        }

    // ---- orientation, area, inscribed radius (user order)
    std::vector<int32_t> tri(3 * nc);
    std::vector<double> area(nc), inr(nc);
    for (int64_t c = 0; c < nc; ++c) {
        int32_t v0 = tri_in[3 * c], v1 = tri_in[3 * c + 1],
                v2 = tri_in[3 * c + 2];
        if (v0 < 0 || v1 < 0 || v2 < 0 || v0 >= nn || v1 >= nn || v2 >= nn) {
            err = fmt("triangle %lld references a node out of range",
                      (long long)c);
            return false;
        }
        if (v0 == v1 || v1 == v2 || v0 == v2) {
            err = fmt("triangle %lld repeats a node", (long long)c);
            return false;
        }
        const double x0 = xy[2 * v0], y0 = xy[2 * v0 + 1];
        const double x1 = xy[2 * v1], y1 = xy[2 * v1 + 1];
        const double x2 = xy[2 * v2], y2 = xy[2 * v2 + 1];
        double twice = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
        if (twice == 0.0) {
            err = fmt("triangle %lld has zero area", (long long)c);
            return false;
        }
        if (twice < 0.0) {
            std::swap(v1, v2);
            twice = -twice;
        }
        tri[3 * c] = v0;
        tri[3 * c + 1] = v1;
        tri[3 * c + 2] = v2;
        area[c] = 0.5 * twice;
        double per = 0.0;
        for (int k = 0; k < 3; ++k) {
            const int32_t p = tri[3 * c + k], q = tri[3 * c + (k + 1) % 3];
            const double dx = xy[2 * q] - xy[2 * p];
            const double dy = xy[2 * q + 1] - xy[2 * p + 1];
            per += std::sqrt(dx * dx + dy * dy);
        }
        inr[c] = 2.0 * area[c] / per;
    }

    // ---- unique edges: bucket the 3 nc sides by their lower node, then
    //      sort each (short) bucket by the higher node
    std::vector<int64_t> start(nn + 1, 0);
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < 3; ++k) {
            const int32_t p = tri[3 * c + k], q = tri[3 * c + (k + 1) % 3];
            ++start[std::min(p, q) + 1];
        }
    for (int64_t n = 0; n < nn; ++n) start[n + 1] += start[n];
    std::vector<int32_t> bucket(3 * nc);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t c = 0; c < nc; ++c)
            for (int k = 0; k < 3; ++k) {
                const int32_t p = tri[3 * c + k], q = tri[3 * c + (k + 1) % 3];
                bucket[fill[std::min(p, q)]++] = int32_t(3 * c + k);
            }
    }
    auto hi_node = [&](int32_t s) {
        const int64_t c = s / 3;
        const int k = s % 3;
        return std::max(tri[3 * c + k], tri[3 * c + (k + 1) % 3]);
    };
    auto fwd = [&](int32_t s) {   // side runs from lower to higher node
        const int64_t c = s / 3;
        const int k = s % 3;
        return tri[3 * c + k] < tri[3 * c + (k + 1) % 3];
    };

    // boundary segments bucketed by their lower node
    std::vector<int64_t> sstart(nn + 1, 0);
    std::vector<int32_t> sbucket(nbnd);
    std::vector<char> sused(nbnd, 0);
    for (int64_t s = 0; s < nbnd; ++s) {
        const int32_t p = bnd_nodes[2 * s], q = bnd_nodes[2 * s + 1];
        if (p < 0 || q < 0 || p >= nn || q >= nn || p == q) {
            err = fmt("boundary segment %lld has invalid nodes", (long long)s);
            return false;
        }
        if (bnd_tag[s] < 0 || bnd_tag[s] >= max_tag) {
            err = fmt("boundary segment %lld has tag %d outside [0,%d)",
                      (long long)s, bnd_tag[s], max_tag);
            return false;
        }
        ++sstart[std::min(p, q) + 1];
    }
    for (int64_t n = 0; n < nn; ++n) sstart[n + 1] += sstart[n];
    {
        std::vector<int64_t> fill(sstart.begin(), sstart.end() - 1);
        for (int64_t s = 0; s < nbnd; ++s) {
            const int32_t p = bnd_nodes[2 * s], q = bnd_nodes[2 * s + 1];
            sbucket[fill[std::min(p, q)]++] = int32_t(s);
        }
    }

    // edge table (global edge ids in (lower node, higher node) order)
    std::vector<int32_t> e_left, e_right, e_tag;   // user cells / -1
    std::vector<int8_t> e_lk;                      // left cell's local side
    std::vector<int32_t> side_edge(3 * nc);        // side -> edge
    e_left.reserve(3 * nc / 2 + nn);
    int64_t nb = 0;
    std::vector<int32_t> tmp;
    for (int64_t a = 0; a < nn; ++a) {
        const int64_t s0 = start[a], s1 = start[a + 1];
        tmp.assign(bucket.begin() + s0, bucket.begin() + s1);
        std::sort(tmp.begin(), tmp.end(), [&](int32_t u, int32_t v) {
            const int32_t bu = hi_node(u), bv = hi_node(v);
            return bu != bv ? bu < bv : u < v;
        });
        for (size_t i = 0; i < tmp.size();) {
            size_t j = i + 1;
            while (j < tmp.size() && hi_node(tmp[j]) == hi_node(tmp[i])) ++j;
            const int32_t b = hi_node(tmp[i]);
            if (j - i > 2) {
                err = fmt("edge (%lld,%d) is shared by more than two triangles",
                          (long long)a, b);
                return false;
            }
            const int32_t e = int32_t(e_left.size());
            if (j - i == 2) {
                if (fwd(tmp[i]) == fwd(tmp[i + 1])) {
                    err = fmt("triangles %d and %d overlap along edge "
                              "(%lld,%d)", tmp[i] / 3, tmp[i + 1] / 3,
                              (long long)a, b);
                    return false;
                }
                const int32_t l = fwd(tmp[i]) ? tmp[i] : tmp[i + 1];
                const int32_t r = fwd(tmp[i]) ? tmp[i + 1] : tmp[i];
                e_left.push_back(l / 3);
                e_lk.push_back(int8_t(l % 3));
                e_right.push_back(r / 3);
                e_tag.push_back(0);
                side_edge[l] = e;
                side_edge[r] = e;
            } else {
                const int32_t l = tmp[i];
                int32_t tag = 0;
                for (int64_t k = sstart[a]; k < sstart[a + 1]; ++k) {
                    const int32_t s = sbucket[k];
                    const int32_t hb = std::max(bnd_nodes[2 * s],
                                                bnd_nodes[2 * s + 1]);
                    if (hb == b) {
                        if (sused[s]) {
                            err = fmt("boundary segment (%lld,%d) listed twice",
                                      (long long)a, b);
                            return false;
                        }
                        sused[s] = 1;
                        tag = bnd_tag[s];
                        break;
                    }
                }
                e_left.push_back(l / 3);
                e_lk.push_back(int8_t(l % 3));
                e_right.push_back(-1);
                e_tag.push_back(tag);
                side_edge[l] = e;
                ++nb;
            }
            i = j;
        }
    }
    for (int64_t s = 0; s < nbnd; ++s)
        if (!sused[s]) {
            // either a duplicate of a used segment or not a boundary edge
            const int32_t p = bnd_nodes[2 * s], q = bnd_nodes[2 * s + 1];
            bool dup = false;
            for (int64_t k = sstart[std::min(p, q)];
                 k < sstart[std::min(p, q) + 1]; ++k) {
                const int32_t t = sbucket[k];
                if (t != s && sused[t] &&
                    std::max(bnd_nodes[2 * t], bnd_nodes[2 * t + 1]) ==
                        std::max(p, q))
                    dup = true;
            }
            err = dup ? fmt("boundary segment (%d,%d) listed twice", p, q)
                      : fmt("boundary segment (%d,%d) is not a boundary edge "
                            "of the mesh", p, q);
            return false;
        }
    const int64_t ne = int64_t(e_left.size());

    // edge geometry from the left cell's counter-clockwise traversal p -> q:
    // L = |q - p|, outward normal (dy, -dx) / L
    std::vector<double> enx(ne), eny(ne), elen(ne);
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t c = e_left[e];
        const int k = e_lk[e];
        const int32_t p = tri[3 * c + k], q = tri[3 * c + (k + 1) % 3];
        const double dx = xy[2 * q] - xy[2 * p];
        const double dy = xy[2 * q + 1] - xy[2 * p + 1];
        const double L = std::sqrt(dx * dx + dy * dy);
        elen[e] = L;
        enx[e] = dy / L;
        eny[e] = -dx / L;
    }
    M.tag_length.assign(max_tag, 0.0);
    for (int64_t e = 0; e < ne; ++e)
        if (e_right[e] < 0) M.tag_length[e_tag[e]] += elen[e];

    // ---- internal cell order: Hilbert curve through the centroids, on a
    //      square lattice covering the bounding box (ties keep user order)
    std::vector<int32_t> order(nc);
    std::iota(order.begin(), order.end(), 0);
    if (reorder && nc > 1) {
        double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY,
               ymax = -INFINITY;
        for (int64_t n = 0; n < nn; ++n) {
            xmin = std::min(xmin, xy[2 * n]);
            xmax = std::max(xmax, xy[2 * n]);
            ymin = std::min(ymin, xy[2 * n + 1]);
            ymax = std::max(ymax, xy[2 * n + 1]);
        }
        const double ext = std::max(xmax - xmin, ymax - ymin);
        const double sc = ext > 0 ? 65535.0 / ext : 0.0;
        std::vector<uint64_t> key(nc);
        for (int64_t c = 0; c < nc; ++c) {
            double cx = 0, cy = 0;
            for (int k = 0; k < 3; ++k) {
                cx += xy[2 * tri[3 * c + k]];
                cy += xy[2 * tri[3 * c + k] + 1];
            }
            cx /= 3.0;
            cy /= 3.0;
            const uint32_t qx = uint32_t(std::min(65535.0, std::max(0.0, (cx - xmin) * sc)));
            const uint32_t qy = uint32_t(std::min(65535.0, std::max(0.0, (cy - ymin) * sc)));
            key[c] = (uint64_t(hilbert_index(qx, qy)) << 32) | uint64_t(c);
        }
        std::sort(key.begin(), key.end());
        for (int64_t i = 0; i < nc; ++i) order[i] = int32_t(key[i] & 0xffffffffu);
    }
    M.user_of_internal = order;
    M.internal_of_user.assign(nc, 0);
    for (int64_t i = 0; i < nc; ++i) M.internal_of_user[order[i]] = int32_t(i);

    M.n_nodes = nn;
    M.n_cells = nc;
    M.n_edges = ne;
    M.n_bnd_edges = nb;
    M.area.resize(nc);
    M.inv_area.resize(nc);
    M.inradius.resize(nc);
    M.min_inradius = INFINITY;
    M.total_area = 0.0;
    for (int64_t i = 0; i < nc; ++i) {
        const int32_t u = order[i];
        M.area[i] = area[u];
        M.inv_area[i] = 1.0 / area[u];
        M.inradius[i] = inr[u];
        M.min_inradius = std::min(M.min_inradius, inr[u]);
        M.total_area += area[u];
    }

    // ---- blocks of block_cells consecutive internal cells and their edges:
    //      edges with both cells in the block first, then edges to another
    //      block, then boundary edges; each group in order of first use
    const int32_t B = block_cells;
    const int64_t nblk = (nc + B - 1) / B;
    M.block_cells = B;
    M.n_blocks = int32_t(nblk);
    M.blk_cell.resize(nblk + 1);
    M.blk_edge.resize(nblk + 1);
    M.slots.assign(nc, 0);
    std::vector<int32_t> stamp(ne, -1), slot_of(ne, 0);
    std::vector<int32_t> inner, halo, bnd;
    M.be_left.reserve(size_t(ne * 1.2) + 16);
    int32_t emax = 0;
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t c0 = b * B, c1 = std::min<int64_t>(nc, c0 + B);
        M.blk_cell[b] = int32_t(c0);
        M.blk_edge[b] = int32_t(M.be_left.size());
        inner.clear();
        halo.clear();
        bnd.clear();
        for (int64_t i = c0; i < c1; ++i) {
            const int32_t u = order[i];
            for (int k = 0; k < 3; ++k) {
                const int32_t e = side_edge[3 * int64_t(u) + k];
                if (stamp[e] == int32_t(b)) continue;
                stamp[e] = int32_t(b);
                if (e_right[e] < 0) {
                    bnd.push_back(e);
                } else {
                    const int64_t il = M.internal_of_user[e_left[e]];
                    const int64_t ir = M.internal_of_user[e_right[e]];
                    const bool both = il >= c0 && il < c1 && ir >= c0 && ir < c1;
                    (both ? inner : halo).push_back(e);
                }
            }
        }
        const int32_t base = int32_t(M.be_left.size());
        int32_t s = 0;
        for (const auto *grp : {&inner, &halo, &bnd})
            for (int32_t e : *grp) {
                slot_of[e] = s++;
                M.be_left.push_back(M.internal_of_user[e_left[e]]);
                M.be_right.push_back(e_right[e] >= 0
                                         ? M.internal_of_user[e_right[e]]
                                         : -1 - e_tag[e]);
                M.be_nx.push_back(enx[e]);
                M.be_ny.push_back(eny[e]);
                M.be_len.push_back(elen[e]);
            }
        emax = std::max(emax, s);
        for (int64_t i = c0; i < c1; ++i) {
            const int32_t u = order[i];
            uint64_t pack = 0;
            for (int k = 0; k < 3; ++k) {
                const int32_t e = side_edge[3 * int64_t(u) + k];
                const uint64_t right = (e_right[e] == u) ? 1u : 0u;
                pack |= (uint64_t(slot_of[e]) | (right << 15)) << (16 * k);
            }
            M.slots[i] = pack;
        }
        (void)base;
    }
    M.blk_cell[nblk] = int32_t(nc);
    M.blk_edge[nblk] = int32_t(M.be_left.size());
    M.max_block_edges = emax;
    if (emax >= (1 << 15)) {
        err = "block edge list too long";
        return false;
    }
    return true;
}

}  // namespace swe
