// partition.cpp -- H-matrix partition of Sec. 3.1: cluster tree by principal component
// bisection (eq. (cluster)) down to leaves of at most b_min elements, block cluster tree
// from the root pair, far-field blocks by the admissibility condition eq. (adm)
//   min(diam(X), diam(Y)) <= eta dist(X, Y),
// with axis-aligned boxes of the element vertices (the supports of the trial functions).
// Readings: split at the median of the projections on the principal axis (ties broken by
// element index), first child = lower half; the axis sign is normalised (largest
// component positive) so that the tree is deterministic.
// Several meshes in one context (components, e.g. the meshes of a batch): the tree first
// splits the list of components in halves down to one component, then bisects each
// component as above; no block couples two components.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "host.hpp"

namespace bem {

namespace {

// Eigenvector of the largest eigenvalue of a symmetric 3x3 matrix (cyclic Jacobi).
void principal_axis(double C[3][3], double v[3])
{
    double A[3][3], Vm[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = C[i][j];
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
        double dia = std::fabs(A[0][0]) + std::fabs(A[1][1]) + std::fabs(A[2][2]);
        if (off <= 1e-15 * dia || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = Vm[k][p], vkq = Vm[k][q];
                    Vm[k][p] = c * vkp - s * vkq;
                    Vm[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int best = 0;
    for (int k = 1; k < 3; ++k)
        if (A[k][k] > A[best][best]) best = k;
    for (int k = 0; k < 3; ++k) v[k] = Vm[k][best];
    int big = 0;
    for (int k = 1; k < 3; ++k)
        if (std::fabs(v[k]) > std::fabs(v[big])) big = k;
    if (v[big] < 0)
        for (int k = 0; k < 3; ++k) v[k] = -v[k];
}

struct Builder {
    const HostGeo& g;
    int leaf;
    Partition& P;

    void box(int node)
    {
        Cluster& c = P.nodes[node];
        for (int k = 0; k < 3; ++k) {
            c.bmin[k] = INFINITY;
            c.bmax[k] = -INFINITY;
        }
        const std::vector<double>* V[3] = {&g.vx, &g.vy, &g.vz};
        for (int t = c.begin; t < c.begin + c.size; ++t) {
            int e = P.perm[t];
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 3; ++k) {
                    double x = (*V[k])[(size_t)a * g.K + e];
                    c.bmin[k] = std::min(c.bmin[k], x);
                    c.bmax[k] = std::max(c.bmax[k], x);
                }
        }
    }

    // element ranges of the components in P.perm (components sorted, contiguous)
    std::vector<int> cbeg;

    // node over the components c0 .. c1 - 1 (more than one)
    int split_comps(int c0, int c1)
    {
        if (c1 - c0 == 1) return split(cbeg[c0], cbeg[c0 + 1] - cbeg[c0], c0);
        int id = (int)P.nodes.size();
        P.nodes.push_back(Cluster{cbeg[c0], cbeg[c1] - cbeg[c0], {-1, -1}, {0, 0, 0}, {0, 0, 0}, -1});
        box(id);
        const int h = (c0 + c1) / 2;
        const int a = split_comps(c0, h);
        const int b = split_comps(h, c1);
        P.nodes[id].child[0] = a;
        P.nodes[id].child[1] = b;
        return id;
    }

    int split(int begin, int size, int comp)
    {
        int id = (int)P.nodes.size();
        P.nodes.push_back(Cluster{begin, size, {-1, -1}, {0, 0, 0}, {0, 0, 0}, comp});
        box(id);
        if (size <= leaf) return id;
        double mu[3] = {0, 0, 0};
        for (int t = begin; t < begin + size; ++t) {
            int e = P.perm[t];
            mu[0] += g.cx[e];
            mu[1] += g.cy[e];
            mu[2] += g.cz[e];
        }
        for (int k = 0; k < 3; ++k) mu[k] /= size;
        double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int t = begin; t < begin + size; ++t) {
            int e = P.perm[t];
            double d[3] = {g.cx[e] - mu[0], g.cy[e] - mu[1], g.cz[e] - mu[2]};
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) C[a][b] += d[a] * d[b];
        }
        double v[3];
        principal_axis(C, v);
        std::vector<std::pair<double, int>> key(size);
        for (int t = 0; t < size; ++t) {
            int e = P.perm[begin + t];
            key[t] = {(g.cx[e] - mu[0]) * v[0] + (g.cy[e] - mu[1]) * v[1] + (g.cz[e] - mu[2]) * v[2], e};
        }
        std::sort(key.begin(), key.end());
        for (int t = 0; t < size; ++t) P.perm[begin + t] = key[t].second;
        int h = size / 2;
        int c0 = split(begin, h, comp);
        int c1 = split(begin + h, size - h, comp);
        P.nodes[id].child[0] = c0;
        P.nodes[id].child[1] = c1;
        return id;
    }

    static double diam(const Cluster& c)
    {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += (c.bmax[k] - c.bmin[k]) * (c.bmax[k] - c.bmin[k]);
        return std::sqrt(s);
    }
    static double dist(const Cluster& a, const Cluster& b)
    {
        double s = 0;
        for (int k = 0; k < 3; ++k) {
            double d = std::max(0.0, std::max(a.bmin[k] - b.bmax[k], b.bmin[k] - a.bmax[k]));
            s += d * d;
        }
        return std::sqrt(s);
    }

    void blocks(int a, int b, double eta)
    {
        const Cluster& A = P.nodes[a];
        const Cluster& B = P.nodes[b];
        if (A.comp >= 0 && B.comp >= 0 && A.comp != B.comp) return;  // two components: no block
        if (A.comp < 0 || B.comp < 0) {  // a node over several components: split it
            if (A.comp < 0) {
                blocks(A.child[0], b, eta);
                blocks(A.child[1], b, eta);
            } else {
                blocks(a, B.child[0], eta);
                blocks(a, B.child[1], eta);
            }
            return;
        }
        if (std::min(diam(A), diam(B)) <= eta * dist(A, B)) {
            P.blocks.push_back(BlockDesc{A.begin, A.size, B.begin, B.size, 1});
            return;
        }
        bool la = A.child[0] < 0, lb = B.child[0] < 0;
        if (la && lb) {
            P.blocks.push_back(BlockDesc{A.begin, A.size, B.begin, B.size, 0});
            return;
        }
        int ca0 = A.child[0], ca1 = A.child[1], cb0 = B.child[0], cb1 = B.child[1];
        if (la) {
            blocks(a, cb0, eta);
            blocks(a, cb1, eta);
        } else if (lb) {
            blocks(ca0, b, eta);
            blocks(ca1, b, eta);
        } else {
            blocks(ca0, cb0, eta);
            blocks(ca0, cb1, eta);
            blocks(ca1, cb0, eta);
            blocks(ca1, cb1, eta);
        }
    }
};

}  // namespace

void build_partition(const HostGeo& g, double eta, int leaf, Partition& out)
{
    out.perm.resize(g.K);
    std::iota(out.perm.begin(), out.perm.end(), 0);
    out.nodes.clear();
    out.blocks.clear();
    Builder B{g, leaf, out, {}};
    if (g.ncomp <= 1 || g.comp.empty()) {
        B.split(0, g.K, 0);
    } else {
        std::stable_sort(out.perm.begin(), out.perm.end(), [&](int x, int y) { return g.comp[x] < g.comp[y]; });
        B.cbeg.assign(g.ncomp + 1, 0);
        for (int e = 0; e < g.K; ++e) ++B.cbeg[g.comp[e] + 1];
        for (int c = 0; c < g.ncomp; ++c) B.cbeg[c + 1] += B.cbeg[c];
        B.split_comps(0, g.ncomp);
    }
    B.blocks(0, 0, eta);
}

}  // namespace bem
