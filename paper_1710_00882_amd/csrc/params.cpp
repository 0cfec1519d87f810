// Parameter files in the LAMMPS "tersoff" format (host code of libtersoff.so;
// declared in include/tersoff.h).
//
// The format is the widely used public one: after '#' comments are removed,
// the file is a stream of entries of 17 words each -- three element names
// (centre i, bond partner j, third atom k) and then m, gamma, lambda3, c, d,
// cos(theta0), n, beta, lambda2, B, R, D, lambda1, A -- in any line layout.
// Entries naming an element outside the requested list are skipped.
#include "tersoff.h"

#include <cerrno>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace {

constexpr int kWords = 17;

std::vector<std::string> words_of(const char *text)
{
    std::vector<std::string> w;
    std::string cur;
    bool comment = false;
    for (const char *p = text; *p; ++p) {
        const char ch = *p;
        if (ch == '\n' || ch == '\r') comment = false;
        if (ch == '#') comment = true;
        const bool space = ch == ' ' || ch == '\t' || ch == '\n' || ch == '\r' || ch == '\f' || ch == '\v';
        if (comment || space) {
            if (!cur.empty()) w.push_back(cur), cur.clear();
            continue;
        }
        cur.push_back(ch);
    }
    if (!cur.empty()) w.push_back(cur);
    return w;
}

bool number(const std::string &s, double &v)
{
    errno = 0;
    char *end = nullptr;
    v = std::strtod(s.c_str(), &end);
    return errno == 0 && end && *end == '\0' && std::isfinite(v);
}

}  // namespace

extern "C" int tersoff_parse_params(const char *text, const char *const *elements, int32_t nelem,
                                    double *params_out)
{
    if (!text || !elements || !params_out || nelem < 1 || nelem > TERSOFF_MAX_TYPES) return TERSOFF_E_INVALID;
    for (int e = 0; e < nelem; ++e)
        if (!elements[e] || !elements[e][0]) return TERSOFF_E_INVALID;
    const std::vector<std::string> w = words_of(text);
    if (w.size() % kWords != 0) return TERSOFF_E_INVALID;
    const int ne = nelem * nelem * nelem;
    std::vector<char> seen((size_t)ne, 0);
    auto type_of = [&](const std::string &name) {
        for (int e = 0; e < nelem; ++e)
            if (name == elements[e]) return e;
        return -1;
    };
    for (size_t base = 0; base < w.size(); base += kWords) {
        const int ti = type_of(w[base]), tj = type_of(w[base + 1]), tk = type_of(w[base + 2]);
        double v[kWords - 3];
        for (int f = 0; f < kWords - 3; ++f)
            if (!number(w[base + 3 + f], v[f])) return TERSOFF_E_INVALID;
        if (ti < 0 || tj < 0 || tk < 0) continue;   // an element not requested
        const int entry = (ti * nelem + tj) * nelem + tk;
        if (seen[entry]) return TERSOFF_E_INVALID;   // the same triplet twice
        seen[entry] = 1;
        // file order: m gamma lambda3 c d cos(theta0) n beta lambda2 B R D lambda1 A
        double *p = params_out + (size_t)entry * TERSOFF_NPARAM;
        p[TERSOFF_P_M] = v[0];
        p[TERSOFF_P_GAMMA] = v[1];
        p[TERSOFF_P_LAMBDA3] = v[2];
        p[TERSOFF_P_C] = v[3];
        p[TERSOFF_P_D] = v[4];
        p[TERSOFF_P_H] = v[5];
        p[TERSOFF_P_ETA] = v[6];
        p[TERSOFF_P_BETA] = v[7];
        p[TERSOFF_P_LAMBDA2] = v[8];
        p[TERSOFF_P_B] = v[9];
        p[TERSOFF_P_R] = v[10];
        p[TERSOFF_P_DC] = v[11];
        p[TERSOFF_P_LAMBDA1] = v[12];
        p[TERSOFF_P_A] = v[13];
    }
    for (int e = 0; e < ne; ++e)
        if (!seen[e]) return TERSOFF_E_INVALID;   // every (ti, tj, tk) is required
    return TERSOFF_OK;
}
