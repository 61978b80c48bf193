// Molecular-surface and charge ingestion (host code): the inputs of the
// paper's solver (Section 2.4, table tb_GPU: the host reads the molecule's
// atom coordinates, radii and charges, and the MSMS triangulation of its
// molecular surface, whose faces and vertices become centroids, normals and
// areas; MSMS is also named in Section 2.1 and 2.2), read into the arrays
// gabi_set_surface_mesh and gabi_set_charges take.
//
// MSMS writes two text files:
//   <name>.vert  comment lines starting with '#', a line whose first field
//                is the vertex count, then one vertex per line:
//                x y z nx ny nz face sphere type  (the vertex normal points
//                out of the molecule)
//   <name>.face  comment lines, a line whose first field is the face count,
//                then one triangle per line: v1 v2 v3 type sphere, with
//                1-based vertex numbers
// A PQR file holds ATOM/HETATM records whose last five fields are
// x y z charge radius (the chain field before them is optional); other
// records are skipped.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/gabi.h"

namespace {

bool skip_line(const std::string &l) {
    for (char c : l) {
        if (c == '#') return true;
        if (c != ' ' && c != '\t' && c != '\r') return false;
    }
    return true;  // blank
}

// Reads the count line and then `fields` numbers per record line.
int read_table(const char *path, int fields, int64_t *count, std::vector<double> *out) {
    if (!path) return GABI_EINVAL;
    std::ifstream f(path);
    if (!f) return GABI_EINVAL;
    std::string line;
    int64_t n = -1;
    while (std::getline(f, line)) {
        if (skip_line(line)) continue;
        std::istringstream ss(line);
        if (!(ss >> n) || n < 0) return GABI_EMESH;
        break;
    }
    if (n < 0) return GABI_EMESH;
    if (count) *count = n;
    if (!out) return GABI_OK;
    out->clear();
    out->reserve((size_t)(n * fields));
    int64_t got = 0;
    while (got < n && std::getline(f, line)) {
        if (skip_line(line)) continue;
        std::istringstream ss(line);
        for (int k = 0; k < fields; ++k) {
            double v;
            if (!(ss >> v) || !std::isfinite(v)) return GABI_EMESH;
            out->push_back(v);
        }
        ++got;
    }
    return got == n ? GABI_OK : GABI_EMESH;
}

bool atom_record(const std::string &l) {
    return l.compare(0, 4, "ATOM") == 0 || l.compare(0, 6, "HETATM") == 0;
}

int read_pqr(const char *path, int64_t cap, int64_t *count, double *xyz, double *q,
             double *radius) {
    if (!path) return GABI_EINVAL;
    std::ifstream f(path);
    if (!f) return GABI_EINVAL;
    std::string line;
    int64_t n = 0;
    while (std::getline(f, line)) {
        if (!atom_record(line)) continue;
        std::istringstream ss(line);
        std::vector<std::string> tok;
        std::string t;
        while (ss >> t) tok.push_back(t);
        if (tok.size() < 6) return GABI_EMESH;
        double v[5];
        for (int k = 0; k < 5; ++k) {
            char *end = nullptr;
            const std::string &s = tok[tok.size() - 5 + k];
            v[k] = std::strtod(s.c_str(), &end);
            if (end == s.c_str() || *end != '\0' || !std::isfinite(v[k])) return GABI_EMESH;
        }
        if (xyz) {
            if (n >= cap) return GABI_EINVAL;
            xyz[3 * n] = v[0];
            xyz[3 * n + 1] = v[1];
            xyz[3 * n + 2] = v[2];
            if (q) q[n] = v[3];
            if (radius) radius[n] = v[4];
        }
        ++n;
    }
    if (count) *count = n;
    return GABI_OK;
}

}  // namespace

extern "C" {

int gabi_msms_counts(const char *vert_path, const char *face_path, int64_t *nv, int64_t *nf) {
    if (!nv || !nf) return GABI_EINVAL;
    int rc = read_table(vert_path, 6, nv, nullptr);
    if (rc) return rc;
    return read_table(face_path, 3, nf, nullptr);
}

int gabi_msms_read(const char *vert_path, const char *face_path, int64_t nv, double *xyz,
                   double *vnormal, int64_t nf, int32_t *tri) {
    if (!xyz || !tri || nv < 3 || nf < 1) return GABI_EINVAL;
    std::vector<double> v, f;
    int64_t cv = 0, cf = 0;
    int rc = read_table(vert_path, 6, &cv, &v);
    if (rc) return rc;
    if ((rc = read_table(face_path, 3, &cf, &f))) return rc;
    if (cv != nv || cf != nf) return GABI_EINVAL;
    for (int64_t i = 0; i < nv; ++i) {
        for (int d = 0; d < 3; ++d) {
            xyz[3 * i + d] = v[(size_t)(6 * i + d)];
            if (vnormal) vnormal[3 * i + d] = v[(size_t)(6 * i + 3 + d)];
        }
    }
    for (int64_t k = 0; k < nf; ++k)
        for (int d = 0; d < 3; ++d) {
            const double one_based = f[(size_t)(3 * k + d)];
            if (one_based != std::floor(one_based) || one_based < 1 || one_based > (double)nv)
                return GABI_EMESH;
            tri[3 * k + d] = (int32_t)one_based - 1;
        }
    return GABI_OK;
}

int gabi_msms_orient(int64_t nv, const double *xyz, const double *vnormal, int64_t nf,
                     int32_t *tri, int64_t *flipped) {
    if (!xyz || !vnormal || !tri || nv < 3 || nf < 1) return GABI_EINVAL;
    int64_t nflip = 0;
    for (int64_t k = 0; k < nf; ++k) {
        const int32_t a = tri[3 * k], b = tri[3 * k + 1], c = tri[3 * k + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) return GABI_EMESH;
        double e1[3], e2[3], s = 0.0;
        for (int d = 0; d < 3; ++d) {
            e1[d] = xyz[3 * b + d] - xyz[3 * a + d];
            e2[d] = xyz[3 * c + d] - xyz[3 * a + d];
        }
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        for (int d = 0; d < 3; ++d)
            s += cr[d] * (vnormal[3 * a + d] + vnormal[3 * b + d] + vnormal[3 * c + d]);
        if (s < 0.0) {  // wound clockwise seen from outside: swap two corners
            tri[3 * k + 1] = c;
            tri[3 * k + 2] = b;
            ++nflip;
        }
    }
    if (flipped) *flipped = nflip;
    return GABI_OK;
}

int gabi_pqr_count(const char *path, int64_t *natoms) {
    if (!natoms) return GABI_EINVAL;
    return read_pqr(path, 0, natoms, nullptr, nullptr, nullptr);
}

int gabi_pqr_read(const char *path, int64_t natoms, double *xyz, double *q, double *radius) {
    if (!xyz || !q) return GABI_EINVAL;
    int64_t n = 0;
    int rc = read_pqr(path, natoms, &n, xyz, q, radius);
    if (rc) return rc;
    return n == natoms ? GABI_OK : GABI_EINVAL;
}

}  // extern "C"
