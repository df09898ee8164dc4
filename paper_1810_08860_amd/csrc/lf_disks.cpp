// Extents of the asymmetric oval disks (Sec. 4.4 of the paper): each disk
// reaches the centres of its 1-ring neighbours in a Delaunay triangulation of
// the disk centres, and its extent towards +u, -u, +v and -v is the furthest
// 1-ring neighbour on that side of the disk's axes. For views on a capture
// sphere the Delaunay triangulation of the centres is the convex hull of their
// directions from the sphere's centre, built here incrementally (a point
// replaces the hull faces it sees by a fan to their horizon). Host code only.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <set>
#include <vector>

#include "../../include/lf.h"
#include "lf_internal.h"

namespace {

int fail(int code, const char *fmt, ...) {
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return lf::fail_msg(code, buf);
}

struct V3 {
    double x, y, z;
};
V3 sub(const V3 &a, const V3 &b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 cross(const V3 &a, const V3 &b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double dot(const V3 &a, const V3 &b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// signed volume: > 0 when d lies on the side of triangle (a, b, c) its
// counter-clockwise normal points to
double orient(const V3 &a, const V3 &b, const V3 &c, const V3 &d) {
    return dot(cross(sub(b, a), sub(c, a)), sub(d, a));
}

struct Face {
    int a, b, c;
    bool alive;
};

// Convex hull of unit vectors p (every point is a vertex); false if the
// points are degenerate (fewer than four not in one plane).
bool hull(const std::vector<V3> &p, std::vector<Face> &faces) {
    const int n = (int)p.size();
    const double eps = 1e-13;
    // a non-degenerate tetrahedron: 0, the point farthest from it, the point
    // farthest from that line, the point farthest from that plane
    int i1 = 0, i2 = -1, i3 = -1;
    double best = 0.0;
    for (int i = 1; i < n; ++i) {
        const V3 d = sub(p[i], p[0]);
        if (dot(d, d) > best) best = dot(d, d), i1 = i;
    }
    if (best < 1e-20) return false;
    best = 0.0;
    for (int i = 0; i < n; ++i) {
        const V3 c = cross(sub(p[i1], p[0]), sub(p[i], p[0]));
        if (dot(c, c) > best) best = dot(c, c), i2 = i;
    }
    if (i2 < 0 || best < 1e-20) return false;
    best = 0.0;
    for (int i = 0; i < n; ++i) {
        const double v = std::fabs(orient(p[0], p[i1], p[i2], p[i]));
        if (v > best) best = v, i3 = i;
    }
    if (i3 < 0 || best < 1e-12) return false;
    int t[4] = {0, i1, i2, i3};
    if (orient(p[t[0]], p[t[1]], p[t[2]], p[t[3]]) > 0.0) std::swap(t[1], t[2]);
    // outward faces of the tetrahedron (the fourth vertex below each)
    faces = {{t[0], t[1], t[2], true}, {t[0], t[3], t[1], true}, {t[1], t[3], t[2], true}, {t[2], t[3], t[0], true}};
    std::vector<char> used(n, 0);
    for (int v : t) used[v] = 1;
    std::vector<int> vis;
    for (int q = 0; q < n; ++q) {
        if (used[q]) continue;
        for (double thr : {eps, -eps}) {  // a point on a face's plane replaces that face
            vis.clear();
            for (int f = 0; f < (int)faces.size(); ++f)
                if (faces[f].alive && orient(p[faces[f].a], p[faces[f].b], p[faces[f].c], p[q]) > thr) vis.push_back(f);
            if (!vis.empty()) break;
        }
        if (vis.empty()) return false;  // a duplicate direction
        // horizon: directed edges of visible faces whose reverse is not one
        std::set<std::pair<int, int>> edges;
        for (int f : vis) {
            const Face &F = faces[f];
            edges.insert({F.a, F.b});
            edges.insert({F.b, F.c});
            edges.insert({F.c, F.a});
        }
        for (int f : vis) faces[f].alive = false;
        for (const auto &e : edges)
            if (!edges.count({e.second, e.first})) faces.push_back({e.first, e.second, q, true});
        used[q] = 1;
    }
    std::vector<Face> out;
    for (const Face &F : faces)
        if (F.alive) out.push_back(F);
    faces.swap(out);
    return (int)faces.size() == 2 * n - 4;  // a closed triangulated sphere with every point a vertex
}

}  // namespace

extern "C" int lf_disk_extents(int32_t n, const double *centres, const double *rot, double scale, double *out_ext) {
    if (!centres || !rot || !out_ext) return fail(LF_EINVAL, "NULL argument");
    if (n < 4 || n > 65535) return fail(LF_EINVAL, "n_views must be in [4, 65535] (got %d)", n);
    if (!(scale > 0.0) || !std::isfinite(scale)) return fail(LF_EINVAL, "scale must be finite and > 0");
    std::vector<V3> p(n);
    for (int i = 0; i < n; ++i) {
        const V3 c{centres[3 * i], centres[3 * i + 1], centres[3 * i + 2]};
        const double r = std::sqrt(dot(c, c));
        if (!(r > 0.0) || !std::isfinite(r)) return fail(LF_EINVAL, "view %d: centre at the origin", i);
        p[i] = {c.x / r, c.y / r, c.z / r};
    }
    std::vector<Face> faces;
    if (!hull(p, faces))
        return fail(LF_EINVAL, "the view directions do not span a closed triangulated sphere");
    std::vector<std::set<int>> ring(n);
    for (const Face &F : faces) {
        ring[F.a].insert({F.b, F.c});
        ring[F.b].insert({F.a, F.c});
        ring[F.c].insert({F.a, F.b});
    }
    for (int i = 0; i < n; ++i) {
        const double *R = rot + 9 * i;  // row-major, columns (r, u, f)
        double e[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j : ring[i]) {
            const double q[3] = {centres[3 * j] - centres[3 * i], centres[3 * j + 1] - centres[3 * i + 1],
                                 centres[3 * j + 2] - centres[3 * i + 2]};
            const double du = q[0] * R[0] + q[1] * R[3] + q[2] * R[6];
            const double dv = q[0] * R[1] + q[1] * R[4] + q[2] * R[7];
            e[0] = std::max(e[0], du);
            e[1] = std::max(e[1], -du);
            e[2] = std::max(e[2], dv);
            e[3] = std::max(e[3], -dv);
        }
        for (int k = 0; k < 4; ++k) {
            if (!(e[k] > 0.0)) return fail(LF_EINVAL, "view %d has no 1-ring neighbour on side %d", i, k);
            out_ext[4 * i + k] = scale * e[k];
        }
    }
    return LF_OK;
}
