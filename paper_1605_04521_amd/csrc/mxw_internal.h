// Internal host-side data structures of the mxw library.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mxw.h"

namespace mxw {

void set_error(const std::string& msg);

// One term of a generator or of its curl: coef * lambda^alpha * vec, where
// vec = grad(lambda_u) for a generator term and grad(lambda_u) x grad(lambda_v)
// for a curl term.
struct Term {
  double coef;
  int8_t alpha[4];
  int8_t u, v;
};

constexpr int kMaxLoc = 45;       // r = 3
constexpr int kMaxFaceLoc = 15;   // r(r+2), r = 3
constexpr int kMaxPhiTerms = 2;
constexpr int kMaxCurlTerms = 7;

// Local generator description on a tet whose local vertices 0..3 are sorted
// by global id.  kind 0 edge / 1 face / 2 volume; entity = local edge or face
// index; sub = index within the entity.
struct LocalGen {
  int kind, entity, sub;
  int i, j;          // edge endpoints (local vertices, i < j)
  int k[4];          // multi-index of weight r-1
};

struct BasisTables {
  int r = 0, nloc = 0, nfloc = 0;
  std::vector<LocalGen> gens;
  // per generator: phi terms then curl terms (padded with coef 0)
  std::vector<Term> phi;    // [nloc][kMaxPhiTerms]
  std::vector<Term> curl;   // [nloc][kMaxCurlTerms]
  int ncurl_max = 0;
  // face-local generators of a face (x<y<z): edges (x,y),(x,z),(y,z) then the
  // face's own generators; expressed with the face's vertices 0,1,2
  std::vector<Term> fphi;   // [nfloc][kMaxPhiTerms]
  // for local face lf of a tet: tet-local generator index of each face-local one
  int face_gen[4][kMaxFaceLoc];
};

BasisTables make_basis(int r);

struct Layout {
  // ---- inputs (copied)
  int64_t nv = 0, nt = 0;
  std::vector<double> xyz;         // [nv][3]
  std::vector<int32_t> tets;       // [nt][4], sorted ascending per tet
  std::vector<double> eps;         // [nt][2]
  std::vector<int32_t> part;       // [nt]
  int32_t n_sub = 0, overlap = 0, r = 1, precision = 0, variant = 0;
  double k0 = 0.0;

  BasisTables basis;

  // ---- entities
  std::vector<std::array<int32_t, 2>> edges;
  std::vector<std::array<int32_t, 3>> faces;
  std::vector<int32_t> tet_edges;  // [nt][6]
  std::vector<int32_t> tet_faces;  // [nt][4]
  std::vector<int32_t> face_t0, face_t1;   // adjacent tets (-1 if none)
  std::vector<int8_t> face_kind;   // -1 interior, MXW_BC_* on the boundary

  // ---- unknowns
  int per_edge = 0, per_face = 0, per_tet = 0;
  int64_t ndof = 0;
  std::vector<int8_t> ent_kind;
  std::vector<int64_t> ent_id;
  std::vector<int16_t> ent_local;
  std::vector<int32_t> tet_dofs;   // [nt][nloc], -1 = eliminated

  // ---- CSR pattern of A
  std::vector<int64_t> rowptr;
  std::vector<int32_t> cols;

  // ---- gather lists for assembly: per global unknown, the entity; per
  // entity (edges, faces, tets in one numbering), its tets and impedance faces
  std::vector<int32_t> dof_ent;          // [ndof] unified entity id
  std::vector<int64_t> ent_tet_ptr;      // [nent+1]
  std::vector<int32_t> ent_tets;
  std::vector<int64_t> ent_imp_ptr;      // [nent+1]
  std::vector<int32_t> ent_imps;         // indices into the face table

  // ---- face table: faces needing B_F (impedance boundary + interface)
  std::vector<int32_t> ft_face;          // face id
  std::vector<int32_t> ft_vert;          // [nft][3] vertex ids ascending
  std::vector<int32_t> ft_dofs;          // [nft][nfloc] global unknowns (-1 eliminated)
  std::vector<int32_t> face_slot;        // face id -> table index or -1
  std::vector<int32_t> imp_ft;           // table indices of impedance boundary faces
  std::vector<int32_t> imp_tet;          // the element adjacent to each impedance face

  // ---- subdomains
  std::vector<int64_t> sub_dof_ptr;      // [n_sub+1]
  std::vector<int32_t> sub_dofs;         // sum n_s, sorted per subdomain
  std::vector<uint8_t> sub_pou;
  std::vector<int64_t> sub_tet_ptr;      // [n_sub+1]
  std::vector<int32_t> sub_tets;
  std::vector<int32_t> sub_lmap;         // [sum |Omega_s|][nloc] local positions
  std::vector<int64_t> sub_face_ptr;     // [n_sub+1]
  std::vector<int32_t> sub_face_ft;      // face table index
  std::vector<int32_t> sub_face_tet;     // element of Omega_s owning the face
  std::vector<uint8_t> sub_face_iface;   // 0 original impedance face, 1 interface face
  std::vector<int32_t> sub_face_lmap;    // [.][nfloc]
  std::vector<int32_t> owner;            // [ndof] owning subdomain
  std::vector<int64_t> owner_pos;        // [ndof] position in the concatenated local vectors
  int64_t n_iface = 0;

  // ---- statistics
  int64_t sum_ns = 0, max_ns = 0;
  double sum_ns2 = 0, sum_ns3 = 0;
};

mxw_status build_layout(const mxw_problem_desc* d, Layout& L);

// beta of each impedance face and the coefficient of each subdomain face
// (beta on original impedance faces, w~ on interface faces; both k0 sqrt(Re eps)
// of the owning element) for a permittivity field eps[nt][2]
void face_coefficients(const Layout& L, const double* eps, double k0, std::vector<double>& imp_beta,
                       std::vector<double>& sub_face_coef);

}  // namespace mxw
