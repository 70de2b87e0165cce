// Degree-r Nedelec generators lambda^k w^e on a tetrahedron (Sec. 3) and their
// symbolic terms, used by the element and face kernels.
//
// Independent subset (the paper defers the choice to other work): for a tet
// with vertices sorted by global id, keep every edge generator; on a face
// x<y<z keep the generators on edges (x,y) (with k_z >= 1) and (x,z) (with
// k_y >= 1); inside the tet (r = 3) keep lambda_c lambda_d w^{ab},
// lambda_b lambda_d w^{ac}, lambda_b lambda_c w^{ad}.  Within an entity the
// multi-index runs in descending lexicographic order.
#include <algorithm>
#include <cstring>

#include "mxw_internal.h"

namespace mxw {
namespace {

const int kEdges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int kFaces[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

int edge_index(int a, int b) {
  for (int e = 0; e < 6; ++e)
    if (kEdges[e][0] == a && kEdges[e][1] == b) return e;
  return -1;
}

// multi-indices of weight s on the vertex list vs (2 or 3 entries), in
// descending lexicographic order of (k_{vs[0]}, k_{vs[1]}, ...)
std::vector<std::array<int, 4>> weights(const std::vector<int>& vs, int s) {
  std::vector<std::array<int, 4>> out;
  if (vs.size() == 2) {
    for (int a = s; a >= 0; --a) {
      std::array<int, 4> k{0, 0, 0, 0};
      k[vs[0]] = a;
      k[vs[1]] = s - a;
      out.push_back(k);
    }
  } else {
    for (int a = s; a >= 0; --a)
      for (int b = s - a; b >= 0; --b) {
        std::array<int, 4> k{0, 0, 0, 0};
        k[vs[0]] = a;
        k[vs[1]] = b;
        k[vs[2]] = s - a - b;
        out.push_back(k);
      }
  }
  return out;
}

Term make_term(double c, const int alpha[4], int u, int v) {
  Term t;
  t.coef = c;
  for (int q = 0; q < 4; ++q) t.alpha[q] = (int8_t)alpha[q];
  t.u = (int8_t)u;
  t.v = (int8_t)v;
  return t;
}

Term zero_term() {
  int z[4] = {0, 0, 0, 0};
  return make_term(0.0, z, 0, 0);
}

// generator terms: lambda^k (lambda_i grad l_j - lambda_j grad l_i)
void phi_terms(const LocalGen& g, Term out[kMaxPhiTerms]) {
  int a1[4], a2[4];
  for (int q = 0; q < 4; ++q) a1[q] = a2[q] = g.k[q];
  a1[g.i] += 1;
  a2[g.j] += 1;
  out[0] = make_term(1.0, a1, g.j, -1);
  out[1] = make_term(-1.0, a2, g.i, -1);
}

// curl terms: grad(lambda^k) x w + 2 lambda^k grad l_i x grad l_j
int curl_terms(const LocalGen& g, Term out[kMaxCurlTerms]) {
  int n = 0;
  auto push = [&](double c, const int al[4], int u, int v) {
    if (u == v || c == 0.0) return;
    if (u > v) {
      std::swap(u, v);
      c = -c;
    }
    out[n++] = make_term(c, al, u, v);
  };
  push(2.0, g.k, g.i, g.j);
  for (int m = 0; m < 4; ++m) {
    if (g.k[m] == 0) continue;
    int b1[4], b2[4];
    for (int q = 0; q < 4; ++q) b1[q] = b2[q] = g.k[q];
    b1[m] -= 1;
    b2[m] -= 1;
    b1[g.i] += 1;   // k_m lambda^{k-e_m} lambda_i (grad l_m x grad l_j)
    b2[g.j] += 1;   // -k_m lambda^{k-e_m} lambda_j (grad l_m x grad l_i)
    push((double)g.k[m], b1, m, g.j);
    push(-(double)g.k[m], b2, m, g.i);
  }
  for (int q = n; q < kMaxCurlTerms; ++q) out[q] = zero_term();
  return n;
}

}  // namespace

BasisTables make_basis(int r) {
  BasisTables B;
  B.r = r;
  // edges
  for (int e = 0; e < 6; ++e) {
    int i = kEdges[e][0], j = kEdges[e][1];
    auto ks = weights({i, j}, r - 1);
    for (size_t s = 0; s < ks.size(); ++s) {
      LocalGen g{0, e, (int)s, i, j, {ks[s][0], ks[s][1], ks[s][2], ks[s][3]}};
      B.gens.push_back(g);
    }
  }
  // faces
  if (r >= 2) {
    for (int f = 0; f < 4; ++f) {
      int x = kFaces[f][0], y = kFaces[f][1], z = kFaces[f][2];
      int s = 0;
      for (auto k : weights({x, y, z}, r - 1))
        if (k[z] >= 1) B.gens.push_back(LocalGen{1, f, s++, x, y, {k[0], k[1], k[2], k[3]}});
      for (auto k : weights({x, y, z}, r - 1))
        if (k[y] >= 1) B.gens.push_back(LocalGen{1, f, s++, x, z, {k[0], k[1], k[2], k[3]}});
    }
  }
  // volume
  if (r == 3) {
    B.gens.push_back(LocalGen{2, 0, 0, 0, 1, {0, 0, 1, 1}});
    B.gens.push_back(LocalGen{2, 0, 1, 0, 2, {0, 1, 0, 1}});
    B.gens.push_back(LocalGen{2, 0, 2, 0, 3, {0, 1, 1, 0}});
  }
  B.nloc = (int)B.gens.size();
  B.phi.resize((size_t)B.nloc * kMaxPhiTerms);
  B.curl.resize((size_t)B.nloc * kMaxCurlTerms);
  for (int p = 0; p < B.nloc; ++p) {
    phi_terms(B.gens[p], &B.phi[(size_t)p * kMaxPhiTerms]);
    int n = curl_terms(B.gens[p], &B.curl[(size_t)p * kMaxCurlTerms]);
    B.ncurl_max = std::max(B.ncurl_max, n);
  }

  // face-local generators: edges (0,1), (0,2), (1,2) of the face, then the
  // face's own generators, with the face's vertices numbered 0,1,2
  std::vector<LocalGen> fg;
  const int fe[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int e = 0; e < 3; ++e)
    for (auto k : weights({fe[e][0], fe[e][1]}, r - 1))
      fg.push_back(LocalGen{0, e, 0, fe[e][0], fe[e][1], {k[0], k[1], k[2], k[3]}});
  if (r >= 2) {
    for (auto k : weights({0, 1, 2}, r - 1))
      if (k[2] >= 1) fg.push_back(LocalGen{1, 0, 0, 0, 1, {k[0], k[1], k[2], k[3]}});
    for (auto k : weights({0, 1, 2}, r - 1))
      if (k[1] >= 1) fg.push_back(LocalGen{1, 0, 0, 0, 2, {k[0], k[1], k[2], k[3]}});
  }
  B.nfloc = (int)fg.size();
  B.fphi.resize((size_t)B.nfloc * kMaxPhiTerms);
  for (int p = 0; p < B.nfloc; ++p) phi_terms(fg[p], &B.fphi[(size_t)p * kMaxPhiTerms]);

  // tet-local generator of each face-local generator, per local face
  for (int lf = 0; lf < 4; ++lf) {
    const int* fv = kFaces[lf];
    int q = 0;
    for (int e = 0; e < 3; ++e) {
      int le = edge_index(fv[fe[e][0]], fv[fe[e][1]]);
      for (int p = 0; p < B.nloc; ++p)
        if (B.gens[p].kind == 0 && B.gens[p].entity == le) B.face_gen[lf][q++] = p;
    }
    for (int p = 0; p < B.nloc; ++p)
      if (B.gens[p].kind == 1 && B.gens[p].entity == lf) B.face_gen[lf][q++] = p;
  }
  return B;
}

}  // namespace mxw
