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

// Stable LSD radix sort of 64-bit keys on bits [lo_bit, 64), 16 bits per
// pass; keys equal on those bits keep their input order.
void radix_sort_u64(std::vector<uint64_t> &a, int lo_bit)
{
    std::vector<uint64_t> tmp(a.size());
    for (int shift = lo_bit; shift < 64; shift += 16) {
        std::vector<size_t> cnt(65537, 0);
        for (uint64_t v : a) ++cnt[((v >> shift) & 0xffffu) + 1];
        bool trivial = false;
        for (size_t d = 0; d < 65536; ++d)
            if (cnt[d + 1] == a.size()) trivial = true;
        if (trivial) continue;
        for (size_t d = 0; d < 65536; ++d) cnt[d + 1] += cnt[d];
        for (uint64_t v : a) tmp[cnt[(v >> shift) & 0xffffu]++] = v;
        a.swap(tmp);
    }
}

// Edge table from a caller's edge list (oriented triangles `tri`). Every
// listed edge must be a side of each triangle it names, no two edges may
// join the same two nodes, every side of every triangle must be on exactly
// one listed edge, and the two triangles of an interior edge must lie on
// opposite sides of it. The left cell of an interior edge is the one whose
// counter-clockwise boundary runs from the lower to the higher node number
// (the order the triangles are listed in does not matter), so the result
// is the edge table the library would discover itself, in the caller's
// edge numbering.
bool edges_from_list(int64_t nn, int64_t nc, const std::vector<int32_t> &tri,
                     const EdgeInput &in, int32_t max_tag,
                     std::vector<int32_t> &e_left, std::vector<int8_t> &e_lk,
                     std::vector<int32_t> &e_right,
                     std::vector<int32_t> &e_tag,
                     std::vector<int32_t> &side_edge, int64_t &nb,
                     std::string &err)
{
    const int64_t ne = in.n;
    if (ne < 0 || ne > INT32_MAX) {
        err = "edge count out of range";
        return false;
    }
    if (ne > 0 && (!in.nodes || !in.cells)) {
        err = "null edge array";
        return false;
    }
    e_left.assign(ne, -1);
    e_lk.assign(ne, 0);
    e_right.assign(ne, -1);
    e_tag.assign(ne, 0);
    side_edge.assign(3 * nc, -1);
    nb = 0;
    // local side of triangle c joining nodes p and q, or -1
    auto side_of = [&](int64_t c, int32_t p, int32_t q) {
        for (int k = 0; k < 3; ++k) {
            const int32_t a = tri[3 * c + k], b = tri[3 * c + (k + 1) % 3];
            if ((a == p && b == q) || (a == q && b == p)) return k;
        }
        return -1;
    };
    std::vector<int32_t> lo_count(nn + 1, 0);
    for (int64_t e = 0; e < ne; ++e) {
        const int32_t p = in.nodes[2 * e], q = in.nodes[2 * e + 1];
        if (p < 0 || q < 0 || p >= nn || q >= nn || p == q) {
            err = fmt("edge %lld has invalid nodes (%d,%d)", (long long)e, p, q);
            return false;
        }
        int32_t cs[2] = {in.cells[2 * e], in.cells[2 * e + 1]};
        if (cs[0] < 0 && cs[1] < 0) {
            err = fmt("edge %lld names no triangle", (long long)e);
            return false;
        }
        if (cs[0] == cs[1]) {
            err = fmt("edge %lld names triangle %d twice", (long long)e, cs[0]);
            return false;
        }
        int ks[2] = {-1, -1};
        for (int j = 0; j < 2; ++j) {
            const int32_t c = cs[j];
            if (c < -1 || c >= nc) {
                err = fmt("edge %lld names triangle %d out of range",
                          (long long)e, c);
                return false;
            }
            if (c < 0) continue;
            ks[j] = side_of(c, p, q);
            if (ks[j] < 0) {
                err = fmt("edge %lld (%d,%d) is not a side of triangle %d",
                          (long long)e, p, q, c);
                return false;
            }
            int32_t &slot = side_edge[3 * int64_t(c) + ks[j]];
            if (slot >= 0) {
                err = fmt("side (%d,%d) of triangle %d is listed by edges %d "
                          "and %lld", p, q, c, slot, (long long)e);
                return false;
            }
            slot = int32_t(e);
        }
        const int32_t tag = in.tag ? in.tag[e] : 0;
        const bool interior = cs[0] >= 0 && cs[1] >= 0;
        if (interior ? tag != 0 : (tag < 0 || tag >= max_tag)) {
            err = interior
                      ? fmt("interior edge %lld carries tag %d (must be 0)",
                            (long long)e, tag)
                      : fmt("boundary edge %lld has tag %d outside [0,%d)",
                            (long long)e, tag, max_tag);
            return false;
        }
        // does side k of triangle c run from the lower to the higher node?
        auto fwd = [&](int32_t c, int k) {
            return tri[3 * int64_t(c) + k] < tri[3 * int64_t(c) + (k + 1) % 3];
        };
        if (interior) {
            if (fwd(cs[0], ks[0]) == fwd(cs[1], ks[1])) {
                err = fmt("triangles %d and %d overlap along edge %lld",
                          cs[0], cs[1], (long long)e);
                return false;
            }
            const int l = fwd(cs[0], ks[0]) ? 0 : 1;
            e_left[e] = cs[l];
            e_lk[e] = int8_t(ks[l]);
            e_right[e] = cs[1 - l];
        } else {
            const int j = cs[0] >= 0 ? 0 : 1;
            e_left[e] = cs[j];
            e_lk[e] = int8_t(ks[j]);
            e_tag[e] = tag;
            ++nb;
        }
        ++lo_count[std::min(p, q) + 1];
    }
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < 3; ++k)
            if (side_edge[3 * c + k] < 0) {
                err = fmt("side %d of triangle %lld is on no listed edge", k,
                          (long long)c);
                return false;
            }
    // no two edges may join the same nodes (a third triangle on a side)
    for (int64_t n = 0; n < nn; ++n) lo_count[n + 1] += lo_count[n];
    std::vector<int32_t> hi(ne);
    {
        std::vector<int32_t> fill(lo_count.begin(), lo_count.end() - 1);
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t p = in.nodes[2 * e], q = in.nodes[2 * e + 1];
            hi[fill[std::min(p, q)]++] = std::max(p, q);
        }
    }
    for (int64_t n = 0; n < nn; ++n) {
        int32_t *b0 = hi.data() + lo_count[n], *b1 = hi.data() + lo_count[n + 1];
        std::sort(b0, b1);
        for (int32_t *x = b0; x + 1 < b1; ++x)
            if (x[0] == x[1]) {
                err = fmt("two edges join nodes %lld and %d", (long long)n,
                          x[0]);
                return false;
            }
    }
    return true;
}

}  // namespace

bool build_block_mesh(int64_t nn, const double *xy, int64_t nc,
                      const int32_t *tri_in, int64_t nbnd,
                      const int32_t *bnd_nodes, const int32_t *bnd_tag,
                      int32_t block_cells, bool reorder,
                      const uint8_t *group, int32_t wet_band,
                      int32_t max_tag, BlockMesh &M, std::string &err,
                      const EdgeInput *edges)
{
    M = BlockMesh();
    if (nn < 3 || nc < 1) {
        err = "mesh needs at least 3 nodes and 1 triangle";
        return false;
    }
    if (nn > INT32_MAX - 1 || nc > INT32_MAX / 3) {
        err = "mesh too large for 32-bit indices";
        return false;
    }
    // the step addresses its 8-byte cell arrays with 32-bit byte offsets
    if (nc >= (int64_t(1) << 29)) {
        err = "mesh too large: fewer than 2^29 cells";
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
    int64_t bad_cell = INT64_MAX;
#pragma omp parallel for schedule(static) reduction(min : bad_cell)
    for (int64_t c = 0; c < nc; ++c) {
        int32_t v0 = tri_in[3 * c], v1 = tri_in[3 * c + 1],
                v2 = tri_in[3 * c + 2];
        if (v0 < 0 || v1 < 0 || v2 < 0 || v0 >= nn || v1 >= nn || v2 >= nn ||
            v0 == v1 || v1 == v2 || v0 == v2) {
            bad_cell = std::min(bad_cell, c);
            continue;
        }
        const double x0 = xy[2 * v0], y0 = xy[2 * v0 + 1];
        const double x1 = xy[2 * v1], y1 = xy[2 * v1 + 1];
        const double x2 = xy[2 * v2], y2 = xy[2 * v2 + 1];
        double twice = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
        if (twice == 0.0) {
            bad_cell = std::min(bad_cell, c);
            continue;
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
    if (bad_cell != INT64_MAX) {
        const int64_t c = bad_cell;
        const int32_t v0 = tri_in[3 * c], v1 = tri_in[3 * c + 1],
                      v2 = tri_in[3 * c + 2];
        if (v0 < 0 || v1 < 0 || v2 < 0 || v0 >= nn || v1 >= nn || v2 >= nn)
            err = fmt("triangle %lld references a node out of range",
                      (long long)c);
        else if (v0 == v1 || v1 == v2 || v0 == v2)
            err = fmt("triangle %lld repeats a node", (long long)c);
        else
            err = fmt("triangle %lld has zero area", (long long)c);
        return false;
    }

    // ---- the edge table: left cell and its side, right cell (-1 on the
    //      boundary), tag, and the edge of every cell side
    std::vector<int32_t> e_left, e_right, e_tag, side_edge;
    std::vector<int8_t> e_lk;
    int64_t ne = 0, nb = 0;
    if (edges) {
        if (!edges_from_list(nn, nc, tri, *edges, max_tag, e_left, e_lk,
                             e_right, e_tag, side_edge, nb, err))
            return false;
        ne = edges->n;
    } else {
        // ---- unique edges: bucket the 3 nc sides by their lower node, then
        //      sort each (short) bucket by (higher node, side)
        std::vector<int64_t> start(nn + 1, 0);
        {
            std::vector<int32_t> cnt(nn, 0);
#pragma omp parallel for schedule(static)
            for (int64_t s = 0; s < 3 * nc; ++s) {
                const int64_t c = s / 3;
                const int k = int(s % 3);
                const int32_t p = tri[3 * c + k], q = tri[3 * c + (k + 1) % 3];
#pragma omp atomic
                cnt[std::min(p, q)] += 1;
            }
            for (int64_t n = 0; n < nn; ++n) start[n + 1] = start[n] + cnt[n];
        }
        std::vector<int32_t> bucket(3 * nc);
        {
            std::vector<int64_t> fill(start.begin(), start.end() - 1);
#pragma omp parallel for schedule(static)
            for (int64_t s = 0; s < 3 * nc; ++s) {
                const int64_t c = s / 3;
                const int k = int(s % 3);
                const int32_t p = tri[3 * c + k], q = tri[3 * c + (k + 1) % 3];
                int64_t at;
#pragma omp atomic capture
                at = fill[std::min(p, q)]++;
                bucket[at] = int32_t(s);
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

        // pass 1: sort each bucket, validate, count its unique edges
        std::vector<int64_t> estart(nn + 1, 0);
        int64_t bad_node = INT64_MAX;
#pragma omp parallel for schedule(dynamic, 4096) reduction(min : bad_node)
        for (int64_t a = 0; a < nn; ++a) {
            int32_t *b0 = bucket.data() + start[a];
            int32_t *b1 = bucket.data() + start[a + 1];
            std::sort(b0, b1, [&](int32_t u, int32_t v) {
                const int32_t bu = hi_node(u), bv = hi_node(v);
                return bu != bv ? bu < bv : u < v;
            });
            int64_t ne_a = 0;
            for (int32_t *i = b0; i < b1;) {
                int32_t *j = i + 1;
                while (j < b1 && hi_node(*j) == hi_node(*i)) ++j;
                if (j - i > 2 || (j - i == 2 && fwd(i[0]) == fwd(i[1])))
                    bad_node = std::min(bad_node, a);
                ++ne_a;
                i = j;
            }
            estart[a + 1] = ne_a;
        }
        if (bad_node != INT64_MAX) {
            const int64_t a = bad_node;
            for (int64_t i = start[a]; i < start[a + 1];) {
                int64_t j = i + 1;
                while (j < start[a + 1] && hi_node(bucket[j]) == hi_node(bucket[i]))
                    ++j;
                const int32_t b = hi_node(bucket[i]);
                if (j - i > 2) {
                    err = fmt("edge (%lld,%d) is shared by more than two triangles",
                              (long long)a, b);
                    return false;
                }
                if (j - i == 2 && fwd(bucket[i]) == fwd(bucket[i + 1])) {
                    err = fmt("triangles %d and %d overlap along edge (%lld,%d)",
                              bucket[i] / 3, bucket[i + 1] / 3, (long long)a, b);
                    return false;
                }
                i = j;
            }
        }
        for (int64_t a = 0; a < nn; ++a) estart[a + 1] += estart[a];
        ne = estart[nn];
        if (ne > INT32_MAX) {
            err = "mesh too large for 32-bit edge indices";
            return false;
        }

        // pass 2: edge table in (lower node, higher node) order
        e_left.resize(ne);
        e_right.resize(ne);
        e_tag.resize(ne);
        e_lk.resize(ne);
        side_edge.resize(3 * nc);
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : nb)
        for (int64_t a = 0; a < nn; ++a) {
            int64_t e = estart[a];
            for (int64_t i = start[a]; i < start[a + 1]; ++e) {
                int64_t j = i + 1;
                while (j < start[a + 1] && hi_node(bucket[j]) == hi_node(bucket[i]))
                    ++j;
                const int32_t b = hi_node(bucket[i]);
                if (j - i == 2) {
                    const int32_t l = fwd(bucket[i]) ? bucket[i] : bucket[i + 1];
                    const int32_t r = fwd(bucket[i]) ? bucket[i + 1] : bucket[i];
                    e_left[e] = l / 3;
                    e_lk[e] = int8_t(l % 3);
                    e_right[e] = r / 3;
                    e_tag[e] = 0;
                    side_edge[l] = int32_t(e);
                    side_edge[r] = int32_t(e);
                } else {
                    const int32_t l = bucket[i];
                    int32_t tag = 0;
                    for (int64_t k = sstart[a]; k < sstart[a + 1]; ++k) {
                        const int32_t s = sbucket[k];
                        if (std::max(bnd_nodes[2 * s], bnd_nodes[2 * s + 1]) == b) {
                            sused[s] = 1;
                            tag = bnd_tag[s];
                            break;
                        }
                    }
                    e_left[e] = l / 3;
                    e_lk[e] = int8_t(l % 3);
                    e_right[e] = -1;
                    e_tag[e] = tag;
                    side_edge[l] = int32_t(e);
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
        std::vector<int64_t>().swap(start);
        std::vector<int32_t>().swap(bucket);
    }

    // edge geometry from the left cell's counter-clockwise traversal p -> q:
    // L = |q - p|, outward normal (dy, -dx) / L
    std::vector<double> enx(ne), eny(ne), elen(ne);
#pragma omp parallel for schedule(static)
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
    // boundary length per tag, summed in (lower node, higher node) order
    // whatever the edge numbering, so the inflow per unit length rounds the
    // same for a discovered and a listed edge table
    M.tag_length.assign(max_tag, 0.0);
    {
        std::vector<std::pair<uint64_t, int32_t>> bnd;
        bnd.reserve(size_t(nb));
        for (int64_t e = 0; e < ne; ++e)
            if (e_right[e] < 0) {
                const int64_t c = e_left[e];
                const int k = e_lk[e];
                const uint32_t p = uint32_t(tri[3 * c + k]);
                const uint32_t q = uint32_t(tri[3 * c + (k + 1) % 3]);
                bnd.emplace_back(uint64_t(std::min(p, q)) << 32 |
                                     uint64_t(std::max(p, q)),
                                 int32_t(e));
            }
        std::sort(bnd.begin(), bnd.end());
        for (const auto &b : bnd) M.tag_length[e_tag[b.second]] += elen[b.second];
    }

    // ---- internal cell order: Hilbert curve through the centroids, on a
    //      square lattice covering the bounding box (ties keep user order)
    std::vector<int32_t> order(nc);
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
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c) {
            double cx = 0, cy = 0;
            for (int k = 0; k < 3; ++k) {
                cx += xy[2 * tri[3 * c + k]];
                cy += xy[2 * tri[3 * c + k] + 1];
            }
            cx /= 3.0;
            cy /= 3.0;
            const uint32_t qx = uint32_t(
                std::min(65535.0, std::max(0.0, (cx - xmin) * sc)));
            const uint32_t qy = uint32_t(
                std::min(65535.0, std::max(0.0, (cy - ymin) * sc)));
            key[c] = (uint64_t(hilbert_index(qx, qy)) << 32) | uint64_t(c);
        }
        radix_sort_u64(key, 32);   // by curve index; ties in user order
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nc; ++i)
            order[i] = int32_t(key[i] & 0xffffffffu);
        // groups in ascending order, each along the curve: with the cells
        // holding water in one group, blocks are wet or dry as a whole
        // except at the seams, and dry blocks cost next to nothing
        // wet mask to groups: 0 wet, 1 dry within wet_band edge-steps of a
        // wet cell, 2 beyond (a multi-source breadth-first sweep over edges)
        std::vector<uint8_t> band_group;
        if (group && wet_band >= 0) {
            std::vector<int32_t> dist(nc, INT32_MAX);
            for (int64_t c = 0; c < nc; ++c)
                if (group[c]) dist[c] = 0;
            for (int32_t k = 0; k < wet_band; ++k)
                for (int64_t e = 0; e < ne; ++e) {
                    const int32_t l = e_left[e], r = e_right[e];
                    if (r < 0) continue;
                    if (dist[l] == k && dist[r] > k + 1) dist[r] = k + 1;
                    if (dist[r] == k && dist[l] > k + 1) dist[l] = k + 1;
                }
            band_group.resize(nc);
            for (int64_t c = 0; c < nc; ++c)
                band_group[c] = dist[c] == 0 ? 0 : dist[c] <= wet_band ? 1 : 2;
            group = band_group.data();
        }
        if (group) {
            std::vector<int64_t> start(257, 0);
            for (int64_t c = 0; c < nc; ++c) ++start[size_t(group[c]) + 1];
            for (int k = 0; k < 256; ++k) start[k + 1] += start[k];
            std::vector<int32_t> by_group(nc);
            for (int64_t i = 0; i < nc; ++i)
                by_group[start[group[order[i]]]++] = order[i];
            order.swap(by_group);
        }
    } else {
        std::iota(order.begin(), order.end(), 0);
    }
    M.user_of_internal = order;
    M.internal_of_user.assign(nc, 0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) M.internal_of_user[order[i]] = int32_t(i);

    M.n_nodes = nn;
    M.n_cells = nc;
    M.n_edges = ne;
    M.n_bnd_edges = nb;
    M.area.resize(nc);
    M.inradius.resize(nc);
    double rmin = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : rmin)
    for (int64_t i = 0; i < nc; ++i) {
        const int32_t u = order[i];
        M.area[i] = area[u];
        M.inradius[i] = inr[u];
        rmin = std::min(rmin, inr[u]);
    }
    M.min_inradius = rmin;
    M.total_area = 0.0;
    for (int64_t i = 0; i < nc; ++i) M.total_area += M.area[i];

    // ---- blocks of block_cells consecutive internal cells and their edges:
    //      edges to another block first (the step kernel prefetches the
    //      neighbour state of the first block_cells edges), then boundary
    //      edges, then edges with both cells in the block; each group in
    //      order of first use (an edge inside the block is first used by its
    //      lower-numbered cell).
    //      Each side of a block edge is encoded as
    //        in the block:  kSideLocal | k << 12 | local cell   (k = the
    //                       cell's side along this edge, 0..2)
    //        other block:   internal cell index (< 2^30)
    //        boundary:      kSideBoundary | boundary slot (right side
    //                       only; slots numbered in block order)
    const int32_t B = block_cells;
    const int64_t nblk = (nc + B - 1) / B;
    // the step addresses its 8-byte cell arrays with 32-bit byte offsets
    if (nc >= (int64_t(1) << 29)) {
        err = "mesh too large: fewer than 2^29 cells";
        return false;
    }
    M.block_cells = B;
    M.n_blocks = int32_t(nblk);
    M.blk_cell.resize(nblk + 1);
    M.blk_edge.assign(nblk + 1, 0);
    const std::vector<int32_t> &iou = M.internal_of_user;
    // edge and neighbour (internal index, -1 on the boundary) of side k of
    // internal cell i, gathered once in internal order
    std::vector<int32_t> side_e(3 * nc), side_nb(3 * nc);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) {
        const int32_t u = order[i];
        for (int k = 0; k < 3; ++k) {
            const int32_t e = side_edge[3 * int64_t(u) + k];
            side_e[3 * i + k] = e;
            side_nb[3 * i + k] =
                e_right[e] < 0 ? -1
                               : iou[e_left[e] == u ? e_right[e] : e_left[e]];
        }
    }
    int32_t emax = 0;
    std::vector<int64_t> blk_bnd(nblk + 1, 0);   // boundary slots per block
    std::vector<int32_t> n_cross(nblk, 0);        // edges to another block
#pragma omp parallel for schedule(static) reduction(max : emax)
    for (int64_t b = 0; b < nblk; ++b) {
        const int64_t c0 = b * B, c1 = std::min<int64_t>(nc, c0 + B);
        int32_t n = 0, nbnd = 0;
        for (int64_t i = c0; i < c1; ++i)
            for (int k = 0; k < 3; ++k) {
                const int64_t j = side_nb[3 * i + k];
                if (j < 0 || j < c0 || j >= c1 || i < j) ++n;
                if (j < 0) ++nbnd;
                else if (j < c0 || j >= c1) ++n_cross[b];
            }
        M.blk_cell[b] = int32_t(c0);
        M.blk_edge[b + 1] = n;
        blk_bnd[b + 1] = nbnd;
        emax = std::max(emax, n);
    }
    M.blk_cell[nblk] = int32_t(nc);
    for (int64_t b = 0; b < nblk; ++b) {
        M.blk_edge[b + 1] += M.blk_edge[b];
        blk_bnd[b + 1] += blk_bnd[b];
    }
    if (blk_bnd[nblk] >= (int64_t(1) << 30)) {
        err = "mesh too large: at most 2^30 boundary edges";
        return false;
    }
    M.bnd_tag.resize(blk_bnd[nblk]);
    M.blk_bnd.assign(4 * size_t(nblk), 0);
    for (int64_t b = 0; b < nblk; ++b) {
        M.blk_bnd[4 * b] = int32_t(blk_bnd[b]);
        M.blk_bnd[4 * b + 1] = M.blk_edge[b] + n_cross[b];
        M.blk_bnd[4 * b + 2] = int32_t(blk_bnd[b + 1] - blk_bnd[b]);
    }
    M.max_block_edges = emax;
    const int64_t nbe = M.blk_edge[nblk];
    // and its 4-byte edge-record arrays likewise
    if (nbe >= (int64_t(1) << 30)) {
        err = "mesh too large: fewer than 2^30 block-edge records";
        return false;
    }
    M.be_a.resize(nbe);
    M.be_b.resize(nbe);
    M.be_nx.resize(nbe);
    M.be_ny.resize(nbe);
    M.be_len.resize(nbe);
#pragma omp parallel
    {
        struct Use { int64_t i; int k; int32_t e; };
        std::vector<Use> grp[3];
#pragma omp for schedule(static)
        for (int64_t b = 0; b < nblk; ++b) {
            const int64_t c0 = b * B, c1 = std::min<int64_t>(nc, c0 + B);
            for (auto &g : grp) g.clear();
            for (int64_t i = c0; i < c1; ++i)
                for (int k = 0; k < 3; ++k) {
                    const int64_t j = side_nb[3 * i + k];
                    const Use use{i, k, side_e[3 * i + k]};
                    if (j < 0) grp[1].push_back(use);
                    else if (j < c0 || j >= c1) grp[0].push_back(use);
                    else if (i < j) grp[2].push_back(use);
                }
            // side code of internal cell j in this block along edge e
            auto local_code = [&](int64_t j, int32_t e) {
                int kk = 0;
                while (side_e[3 * j + kk] != e) ++kk;
                return int32_t(kSideLocal | (uint32_t(kk) << 12) |
                               uint32_t(j - c0));
            };
            int64_t at = M.blk_edge[b], slot = blk_bnd[b];
            for (int g = 0; g < 3; ++g)
                for (const Use &use : grp[g]) {
                    const int32_t e = use.e;
                    const int64_t il = iou[e_left[e]];
                    const bool l_in = il >= c0 && il < c1;
                    M.be_a[at] = l_in ? local_code(il, e) : int32_t(il);
                    if (e_right[e] < 0) {
                        M.be_b[at] = int32_t(kSideBoundary | uint32_t(slot));
                        M.bnd_tag[slot++] = e_tag[e];
                    } else {
                        const int64_t ir = iou[e_right[e]];
                        const bool r_in = ir >= c0 && ir < c1;
                        M.be_b[at] = r_in ? local_code(ir, e) : int32_t(ir);
                    }
                    M.be_nx[at] = enx[e];
                    M.be_ny[at] = eny[e];
                    M.be_len[at] = elen[e];
                    ++at;
                }
        }
    }

    return true;
}

}  // namespace swe
