// Host-side setup: validation, mesh entities, global unknown numbering,
// sparsity pattern, gather lists for deterministic assembly, and the
// overlapping subdomains with their partition of unity and interface faces.
//
// Numbering (Sec. 3-4; "an ordered set of the unknowns of the whole domain"):
// edges are the distinct sorted vertex pairs in lexicographic order, faces the
// distinct sorted vertex triples in lexicographic order, elements keep input
// order; unknowns run over edges, then faces, then elements; unknowns of
// entities on metallic faces (eq. (2)) are removed keeping relative order.
//
// Overlap: each layer adds the elements that share a face with the current
// subdomain.  Partition of unity (Sec. 4 only requires sum R^T D R = I): an
// unknown belongs to the smallest core id among the elements containing its
// entity, D_s = 1 there and 0 elsewhere.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <sstream>

#include "mxw_internal.h"

namespace mxw {
namespace {

const int kEdges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
const int kFaces[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};

mxw_status fail(const std::string& m) {
  set_error(m);
  return MXW_EINVAL;
}

template <class T>
int64_t find_sorted(const std::vector<T>& v, const T& key) {
  auto it = std::lower_bound(v.begin(), v.end(), key);
  if (it == v.end() || !(*it == key)) return -1;
  return it - v.begin();
}

}  // namespace

mxw_status build_layout(const mxw_problem_desc* d, Layout& L) {
  if (!d) return fail("desc is NULL");
  if (d->n_vertices <= 0 || d->n_tets <= 0 || !d->xyz || !d->tets || !d->eps || !d->part)
    return fail("mesh arrays missing or empty");
  if (d->degree < 1 || d->degree > 3) return fail("degree must be 1, 2 or 3");
  if (d->n_sub < 1) return fail("n_sub must be >= 1");
  if (d->overlap_layers < 0) return fail("overlap_layers must be >= 0");
  if (!(std::isfinite(d->k0)) || d->k0 < 0) return fail("k0 must be finite and >= 0");
  if (d->precision != MXW_FP64 && d->precision != MXW_MIXED) return fail("unknown precision");
  if (d->prec_variant < 0 || d->prec_variant > MXW_PREC_ORAS_MULT) return fail("unknown preconditioner variant");
  if (d->n_vertices >= (int64_t)1 << 31 || d->n_tets >= (int64_t)1 << 31)
    return fail("mesh too large for 32-bit ids");
  if (d->n_bfaces > 0 && (!d->bfaces || !d->bface_kind)) return fail("boundary face arrays missing");

  L.nv = d->n_vertices;
  L.nt = d->n_tets;
  L.n_sub = d->n_sub;
  L.overlap = d->overlap_layers;
  L.r = d->degree;
  L.k0 = d->k0;
  L.precision = d->precision;
  L.variant = d->prec_variant;
  L.basis = make_basis(L.r);
  const int nloc = L.basis.nloc;
  const int64_t nt = L.nt, nv = L.nv;

  L.xyz.assign(d->xyz, d->xyz + 3 * nv);
  for (double x : L.xyz)
    if (!std::isfinite(x)) return fail("non-finite vertex coordinate");
  L.eps.assign(d->eps, d->eps + 2 * nt);
  for (double x : L.eps)
    if (!std::isfinite(x)) return fail("non-finite permittivity");
  L.part.assign(d->part, d->part + nt);
  for (int64_t t = 0; t < nt; ++t)
    if (L.part[t] < 0 || L.part[t] >= L.n_sub) return fail("part id out of range");

  // tets with vertices sorted ascending (local order = global order)
  L.tets.resize(4 * nt);
  for (int64_t t = 0; t < nt; ++t) {
    int32_t v[4];
    for (int q = 0; q < 4; ++q) {
      v[q] = d->tets[4 * t + q];
      if (v[q] < 0 || v[q] >= nv) {
        std::ostringstream os;
        os << "tet " << t << " has a vertex id out of range";
        return fail(os.str());
      }
    }
    std::sort(v, v + 4);
    if (v[0] == v[1] || v[1] == v[2] || v[2] == v[3]) return fail("tet with repeated vertex");
    const double* X0 = &L.xyz[3 * v[0]];
    double e[3][3];
    for (int q = 0; q < 3; ++q)
      for (int c = 0; c < 3; ++c) e[q][c] = L.xyz[3 * v[q + 1] + c] - X0[c];
    double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                 e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                 e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    if (!(std::fabs(det) > 0)) {
      std::ostringstream os;
      os << "tet " << t << " has zero volume";
      return fail(os.str());
    }
    for (int q = 0; q < 4; ++q) L.tets[4 * t + q] = v[q];
  }

  // ---- edges
  {
    std::vector<std::array<int32_t, 2>> all(6 * nt);
    for (int64_t t = 0; t < nt; ++t)
      for (int e = 0; e < 6; ++e)
        all[6 * t + e] = {L.tets[4 * t + kEdges[e][0]], L.tets[4 * t + kEdges[e][1]]};
    L.edges = all;
    std::sort(L.edges.begin(), L.edges.end());
    L.edges.erase(std::unique(L.edges.begin(), L.edges.end()), L.edges.end());
    L.tet_edges.resize(6 * nt);
    for (int64_t q = 0; q < 6 * nt; ++q) L.tet_edges[q] = (int32_t)find_sorted(L.edges, all[q]);
  }
  // ---- faces
  {
    std::vector<std::array<int32_t, 3>> all(4 * nt);
    for (int64_t t = 0; t < nt; ++t)
      for (int f = 0; f < 4; ++f)
        all[4 * t + f] = {L.tets[4 * t + kFaces[f][0]], L.tets[4 * t + kFaces[f][1]],
                          L.tets[4 * t + kFaces[f][2]]};
    L.faces = all;
    std::sort(L.faces.begin(), L.faces.end());
    L.faces.erase(std::unique(L.faces.begin(), L.faces.end()), L.faces.end());
    L.tet_faces.resize(4 * nt);
    for (int64_t q = 0; q < 4 * nt; ++q) L.tet_faces[q] = (int32_t)find_sorted(L.faces, all[q]);
  }
  const int64_t ne = L.edges.size(), nf = L.faces.size();
  L.face_t0.assign(nf, -1);
  L.face_t1.assign(nf, -1);
  for (int64_t t = 0; t < nt; ++t)
    for (int f = 0; f < 4; ++f) {
      int32_t id = L.tet_faces[4 * t + f];
      if (L.face_t0[id] < 0)
        L.face_t0[id] = (int32_t)t;
      else if (L.face_t1[id] < 0)
        L.face_t1[id] = (int32_t)t;
      else
        return fail("a face is shared by more than two tets");
    }
  // ---- boundary faces: must be exactly the faces with one tet
  L.face_kind.assign(nf, -1);
  int64_t nb_mesh = 0;
  for (int64_t f = 0; f < nf; ++f) nb_mesh += (L.face_t1[f] < 0);
  if (d->n_bfaces != nb_mesh) {
    std::ostringstream os;
    os << "boundary faces given: " << d->n_bfaces << ", faces with one tet: " << nb_mesh;
    return fail(os.str());
  }
  for (int64_t b = 0; b < d->n_bfaces; ++b) {
    std::array<int32_t, 3> k = {d->bfaces[3 * b], d->bfaces[3 * b + 1], d->bfaces[3 * b + 2]};
    std::sort(k.begin(), k.end());
    int64_t f = find_sorted(L.faces, k);
    if (f < 0 || L.face_t1[f] >= 0) return fail("a boundary face is not a face with one tet");
    if (L.face_kind[f] >= 0) return fail("duplicate boundary face");
    int kind = d->bface_kind[b];
    if (kind != MXW_BC_PEC && kind != MXW_BC_IMPEDANCE) return fail("unknown boundary kind");
    L.face_kind[f] = (int8_t)kind;
  }

  // ---- unknowns
  const int r = L.r;
  L.per_edge = r;
  L.per_face = r * (r - 1);
  L.per_tet = r * (r - 1) * (r - 2) / 2;
  std::vector<uint8_t> pec_edge(ne, 0), pec_face(nf, 0);
  for (int64_t f = 0; f < nf; ++f)
    if (L.face_kind[f] == MXW_BC_PEC) {
      pec_face[f] = 1;
      const auto& v = L.faces[f];
      const std::array<int32_t, 2> es[3] = {{v[0], v[1]}, {v[0], v[2]}, {v[1], v[2]}};
      for (auto& e : es) pec_edge[find_sorted(L.edges, e)] = 1;
    }
  const int64_t face_base = ne * L.per_edge, tet_base = face_base + nf * L.per_face;
  const int64_t nfull = tet_base + nt * L.per_tet;
  std::vector<int32_t> full_to_dof(nfull, -1);
  int64_t nd = 0;
  L.ent_kind.clear();
  L.ent_id.clear();
  L.ent_local.clear();
  auto add_dof = [&](int64_t full, int kind, int64_t id, int loc) {
    full_to_dof[full] = (int32_t)nd++;
    L.ent_kind.push_back((int8_t)kind);
    L.ent_id.push_back(id);
    L.ent_local.push_back((int16_t)loc);
  };
  for (int64_t e = 0; e < ne; ++e)
    if (!pec_edge[e])
      for (int l = 0; l < L.per_edge; ++l) add_dof(e * L.per_edge + l, 0, e, l);
  for (int64_t f = 0; f < nf; ++f)
    if (!pec_face[f])
      for (int l = 0; l < L.per_face; ++l) add_dof(face_base + f * L.per_face + l, 1, f, l);
  for (int64_t t = 0; t < nt; ++t)
    for (int l = 0; l < L.per_tet; ++l) add_dof(tet_base + t * L.per_tet + l, 2, t, l);
  if (nd >= ((int64_t)1 << 31)) return fail("too many unknowns for 32-bit column ids");
  L.ndof = nd;

  L.tet_dofs.resize((size_t)nt * nloc);
  for (int64_t t = 0; t < nt; ++t)
    for (int p = 0; p < nloc; ++p) {
      const LocalGen& g = L.basis.gens[p];
      int64_t full;
      if (g.kind == 0)
        full = (int64_t)L.tet_edges[6 * t + g.entity] * L.per_edge + g.sub;
      else if (g.kind == 1)
        full = face_base + (int64_t)L.tet_faces[4 * t + g.entity] * L.per_face + g.sub;
      else
        full = tet_base + t * L.per_tet + g.sub;
      L.tet_dofs[(size_t)t * nloc + p] = full_to_dof[full];
    }

  // ---- unified entity numbering (edges, faces, tets) and entity -> tets
  const int64_t nent = ne + nf + nt;
  L.dof_ent.resize(nd);
  for (int64_t i = 0; i < nd; ++i)
    L.dof_ent[i] = (int32_t)(L.ent_kind[i] == 0 ? L.ent_id[i]
                             : L.ent_kind[i] == 1 ? ne + L.ent_id[i]
                                                  : ne + nf + L.ent_id[i]);
  {
    std::vector<int64_t> cnt(nent + 1, 0);
    for (int64_t t = 0; t < nt; ++t) {
      for (int e = 0; e < 6; ++e) cnt[L.tet_edges[6 * t + e] + 1]++;
      for (int f = 0; f < 4; ++f) cnt[ne + L.tet_faces[4 * t + f] + 1]++;
      cnt[ne + nf + t + 1]++;
    }
    for (int64_t q = 0; q < nent; ++q) cnt[q + 1] += cnt[q];
    L.ent_tet_ptr = cnt;
    L.ent_tets.resize(cnt[nent]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < nt; ++t) {   // ascending t -> lists sorted
      for (int e = 0; e < 6; ++e) L.ent_tets[pos[L.tet_edges[6 * t + e]]++] = (int32_t)t;
      for (int f = 0; f < 4; ++f) L.ent_tets[pos[ne + L.tet_faces[4 * t + f]]++] = (int32_t)t;
      L.ent_tets[pos[ne + nf + t]++] = (int32_t)t;
    }
  }

  // ---- CSR pattern: columns of an entity's rows = unknowns of its tets
  {
    std::vector<int64_t> ent_ncol(nent, 0);
    std::vector<std::vector<int32_t>> dummy;
    // pass 1: count columns per entity
    std::vector<int32_t> buf;
    std::vector<int64_t> ent_col_ptr(nent + 1, 0);
    std::vector<int32_t> ent_cols;
    ent_cols.reserve((size_t)nd * 16);
    for (int64_t en = 0; en < nent; ++en) {
      buf.clear();
      for (int64_t q = L.ent_tet_ptr[en]; q < L.ent_tet_ptr[en + 1]; ++q) {
        const int32_t* td = &L.tet_dofs[(size_t)L.ent_tets[q] * nloc];
        for (int p = 0; p < nloc; ++p)
          if (td[p] >= 0) buf.push_back(td[p]);
      }
      std::sort(buf.begin(), buf.end());
      buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
      ent_cols.insert(ent_cols.end(), buf.begin(), buf.end());
      ent_col_ptr[en + 1] = ent_cols.size();
    }
    L.rowptr.assign(nd + 1, 0);
    for (int64_t i = 0; i < nd; ++i) {
      int64_t en = L.dof_ent[i];
      L.rowptr[i + 1] = L.rowptr[i] + (ent_col_ptr[en + 1] - ent_col_ptr[en]);
    }
    L.cols.resize(L.rowptr[nd]);
    for (int64_t i = 0; i < nd; ++i) {
      int64_t en = L.dof_ent[i];
      std::copy(ent_cols.begin() + ent_col_ptr[en], ent_cols.begin() + ent_col_ptr[en + 1],
                L.cols.begin() + L.rowptr[i]);
    }
  }

  // ---- subdomains: overlap growth, N_s, owners, interface faces
  const int nfloc = L.basis.nfloc;
  L.face_slot.assign(nf, -1);
  auto slot_of = [&](int32_t f) {
    if (L.face_slot[f] < 0) {
      L.face_slot[f] = (int32_t)L.ft_face.size();
      L.ft_face.push_back(f);
    }
    return L.face_slot[f];
  };
  // impedance boundary faces first, in face order
  for (int64_t f = 0; f < nf; ++f)
    if (L.face_kind[f] == MXW_BC_IMPEDANCE) {
      int32_t s = slot_of((int32_t)f);
      L.imp_ft.push_back(s);
      L.imp_tet.push_back(L.face_t0[f]);
    }

  L.owner.assign(nd, INT32_MAX);
  for (int64_t t = 0; t < nt; ++t)
    for (int p = 0; p < nloc; ++p) {
      int32_t dd = L.tet_dofs[(size_t)t * nloc + p];
      if (dd >= 0) L.owner[dd] = std::min(L.owner[dd], L.part[t]);
    }

  std::vector<std::vector<int32_t>> core(L.n_sub);
  for (int64_t t = 0; t < nt; ++t) core[L.part[t]].push_back((int32_t)t);
  std::vector<int32_t> mark(nt, -1);
  L.sub_dof_ptr.assign(L.n_sub + 1, 0);
  L.sub_tet_ptr.assign(L.n_sub + 1, 0);
  L.sub_face_ptr.assign(L.n_sub + 1, 0);
  L.sub_dofs.clear();
  L.sub_pou.clear();
  L.sub_tets.clear();
  L.sub_lmap.clear();
  L.owner_pos.assign(nd, -1);
  std::vector<int32_t> set, frontier, next, ldofs;
  for (int32_t s = 0; s < L.n_sub; ++s) {
    set = core[s];
    for (int32_t t : set) mark[t] = s;
    frontier = set;
    for (int layer = 0; layer < L.overlap; ++layer) {
      next.clear();
      for (int32_t t : frontier)
        for (int f = 0; f < 4; ++f) {
          int32_t fid = L.tet_faces[4 * (int64_t)t + f];
          int32_t u = L.face_t0[fid] == t ? L.face_t1[fid] : L.face_t0[fid];
          if (u >= 0 && mark[u] != s) {
            mark[u] = s;
            next.push_back(u);
          }
        }
      set.insert(set.end(), next.begin(), next.end());
      frontier.swap(next);
    }
    std::sort(set.begin(), set.end());
    ldofs.clear();
    for (int32_t t : set)
      for (int p = 0; p < nloc; ++p) {
        int32_t dd = L.tet_dofs[(size_t)t * nloc + p];
        if (dd >= 0) ldofs.push_back(dd);
      }
    std::sort(ldofs.begin(), ldofs.end());
    ldofs.erase(std::unique(ldofs.begin(), ldofs.end()), ldofs.end());
    const int64_t base = L.sub_dofs.size();
    for (size_t q = 0; q < ldofs.size(); ++q) {
      int32_t dd = ldofs[q];
      L.sub_dofs.push_back(dd);
      bool own = L.owner[dd] == s;
      L.sub_pou.push_back(own ? 1 : 0);
      if (own) L.owner_pos[dd] = base + (int64_t)q;
    }
    L.sub_dof_ptr[s + 1] = L.sub_dofs.size();
    for (int32_t t : set) {
      L.sub_tets.push_back(t);
      for (int p = 0; p < nloc; ++p) {
        int32_t dd = L.tet_dofs[(size_t)t * nloc + p];
        L.sub_lmap.push_back(dd < 0 ? -1 : (int32_t)(std::lower_bound(ldofs.begin(), ldofs.end(), dd) - ldofs.begin()));
      }
    }
    L.sub_tet_ptr[s + 1] = L.sub_tets.size();
    // faces: original impedance faces of Omega_s, then interface faces
    for (int pass = 0; pass < 2; ++pass)
      for (int32_t t : set)
        for (int f = 0; f < 4; ++f) {
          int32_t fid = L.tet_faces[4 * (int64_t)t + f];
          int32_t u = L.face_t0[fid] == t ? L.face_t1[fid] : L.face_t0[fid];
          if (pass == 0) {
            if (L.face_kind[fid] != MXW_BC_IMPEDANCE) continue;
          } else {
            if (u < 0 || mark[u] == s) continue;
            L.n_iface++;
          }
          int32_t slot = slot_of(fid);
          L.sub_face_ft.push_back(slot);
          L.sub_face_tet.push_back(t);
          L.sub_face_iface.push_back((uint8_t)pass);
          // face-local unknowns: edges (a,b), (a,c), (b,c), then the face's own
          const auto& v = L.faces[fid];
          std::array<int32_t, 2> es[3] = {{v[0], v[1]}, {v[0], v[2]}, {v[1], v[2]}};
          std::vector<int32_t> gd;
          for (auto& e : es) {
            int64_t eid = find_sorted(L.edges, e);
            for (int l = 0; l < L.per_edge; ++l) gd.push_back(full_to_dof[eid * L.per_edge + l]);
          }
          for (int l = 0; l < L.per_face; ++l) gd.push_back(full_to_dof[face_base + (int64_t)fid * L.per_face + l]);
          for (int q = 0; q < nfloc; ++q)
            L.sub_face_lmap.push_back(gd[q] < 0 ? -1 : (int32_t)(std::lower_bound(ldofs.begin(), ldofs.end(), gd[q]) - ldofs.begin()));
        }
    L.sub_face_ptr[s + 1] = L.sub_face_ft.size();
    const int64_t ns = (int64_t)ldofs.size();
    L.sum_ns += ns;
    L.max_ns = std::max(L.max_ns, ns);
    L.sum_ns2 += (double)ns * ns;
    L.sum_ns3 += (double)ns * ns * ns;
  }
  for (int64_t i = 0; i < nd; ++i)
    if (L.owner_pos[i] < 0) return fail("internal: unknown without owner subdomain");

  // ---- face table: vertices and global unknowns of each face
  const int64_t nft = L.ft_face.size();
  L.ft_vert.resize(3 * nft);
  L.ft_dofs.resize((size_t)nft * nfloc);
  for (int64_t q = 0; q < nft; ++q) {
    const auto& v = L.faces[L.ft_face[q]];
    for (int c = 0; c < 3; ++c) L.ft_vert[3 * q + c] = v[c];
    std::array<int32_t, 2> es[3] = {{v[0], v[1]}, {v[0], v[2]}, {v[1], v[2]}};
    int k = 0;
    for (auto& e : es) {
      int64_t eid = find_sorted(L.edges, e);
      for (int l = 0; l < L.per_edge; ++l) L.ft_dofs[q * nfloc + k++] = full_to_dof[eid * L.per_edge + l];
    }
    for (int l = 0; l < L.per_face; ++l)
      L.ft_dofs[q * nfloc + k++] = full_to_dof[face_base + (int64_t)L.ft_face[q] * L.per_face + l];
  }
  // entity -> impedance faces (for the rows of A)
  {
    std::vector<int64_t> cnt(nent + 1, 0);
    for (size_t q = 0; q < L.imp_ft.size(); ++q) {
      int32_t fid = L.ft_face[L.imp_ft[q]];
      const auto& v = L.faces[fid];
      std::array<int32_t, 2> es[3] = {{v[0], v[1]}, {v[0], v[2]}, {v[1], v[2]}};
      for (auto& e : es) cnt[find_sorted(L.edges, e) + 1]++;
      cnt[ne + fid + 1]++;
    }
    for (int64_t q = 0; q < nent; ++q) cnt[q + 1] += cnt[q];
    L.ent_imp_ptr = cnt;
    L.ent_imps.resize(cnt[nent]);
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (size_t q = 0; q < L.imp_ft.size(); ++q) {
      int32_t fid = L.ft_face[L.imp_ft[q]];
      const auto& v = L.faces[fid];
      std::array<int32_t, 2> es[3] = {{v[0], v[1]}, {v[0], v[2]}, {v[1], v[2]}};
      for (auto& e : es) L.ent_imps[pos[find_sorted(L.edges, e)]++] = (int32_t)q;
      L.ent_imps[pos[ne + fid]++] = (int32_t)q;
    }
  }
  return MXW_OK;
}

void face_coefficients(const Layout& L, const double* eps, double k0, std::vector<double>& imp_beta,
                       std::vector<double>& sub_face_coef) {
  auto wavenumber = [&](int64_t t) { return k0 * std::sqrt(std::max(0.0, eps[2 * t])); };
  imp_beta.resize(L.imp_tet.size());
  for (size_t q = 0; q < L.imp_tet.size(); ++q) imp_beta[q] = wavenumber(L.imp_tet[q]);
  sub_face_coef.resize(L.sub_face_tet.size());
  for (size_t q = 0; q < L.sub_face_tet.size(); ++q) sub_face_coef[q] = wavenumber(L.sub_face_tet[q]);
}

}  // namespace mxw
