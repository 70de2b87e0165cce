// Host-only driver of the library's setup code (unknown numbering, CSR
// pattern, overlapping subdomains, face coefficients), built with g++ and the
// address and undefined-behaviour sanitizers by tests/test_host_sanitize.py.
//
// Usage: layout_check <dir>.  <dir>/meta.txt holds
//   n_vertices n_tets n_bfaces n_sub overlap degree precision variant
// and <dir> holds k0.bin (one f64) and the raw little-endian arrays xyz.bin
// (f64 [nv][3]), tets.bin (i32 [nt][4]), eps.bin (f64 [nt][2]), bfaces.bin
// (i32 [nb][3]), bkind.bin (i8 [nb]) and part.bin (i32 [nt]).  The driver
// writes status.txt (status code, then the error message or "ok") and, on
// success, info.txt and the arrays the library exports, plus the face
// coefficients for the given permittivity.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <iostream>
#include <string>
#include <vector>

#include "../../paper_1605_04521_amd/csrc/mxw_internal.h"

namespace mxw {
static std::string g_error;
void set_error(const std::string& msg) { g_error = msg; }
}  // namespace mxw

template <class T>
static std::vector<T> load(const std::string& path, size_t count) {
  std::vector<T> v(count);
  if (count == 0) return v;
  std::ifstream f(path, std::ios::binary);
  if (!f || !f.read(reinterpret_cast<char*>(v.data()), (std::streamsize)(count * sizeof(T)))) {
    std::cerr << "cannot read " << count << " items from " << path << "\n";
    std::exit(2);
  }
  return v;
}

template <class T>
static void save(const std::string& path, const T* p, size_t count) {
  std::ofstream f(path, std::ios::binary);
  if (count) f.write(reinterpret_cast<const char*>(p), (std::streamsize)(count * sizeof(T)));
  if (!f) {
    std::cerr << "cannot write " << path << "\n";
    std::exit(2);
  }
}

template <class T>
static void save(const std::string& path, const std::vector<T>& v) {
  save(path, v.data(), v.size());
}

int main(int argc, char** argv) {
  if (argc != 2) {
    std::cerr << "usage: layout_check <dir>\n";
    return 2;
  }
  const std::string dir = argv[1];
  std::ifstream meta(dir + "/meta.txt");
  int64_t nv, nt, nb;
  int32_t n_sub, overlap, degree, precision, variant;
  if (!(meta >> nv >> nt >> nb >> n_sub >> overlap >> degree >> precision >> variant)) {
    std::cerr << "bad meta.txt\n";
    return 2;
  }
  const double k0 = load<double>(dir + "/k0.bin", 1)[0];
  const auto xyz = load<double>(dir + "/xyz.bin", (size_t)std::max<int64_t>(nv, 0) * 3);
  const auto tets = load<int32_t>(dir + "/tets.bin", (size_t)std::max<int64_t>(nt, 0) * 4);
  const auto eps = load<double>(dir + "/eps.bin", (size_t)std::max<int64_t>(nt, 0) * 2);
  const auto bfaces = load<int32_t>(dir + "/bfaces.bin", (size_t)std::max<int64_t>(nb, 0) * 3);
  const auto bkind = load<int8_t>(dir + "/bkind.bin", (size_t)std::max<int64_t>(nb, 0));
  const auto part = load<int32_t>(dir + "/part.bin", (size_t)std::max<int64_t>(nt, 0));

  mxw_problem_desc d{};
  d.n_vertices = nv;
  d.xyz = xyz.empty() ? nullptr : xyz.data();
  d.n_tets = nt;
  d.tets = tets.empty() ? nullptr : tets.data();
  d.eps = eps.empty() ? nullptr : eps.data();
  d.n_bfaces = nb;
  d.bfaces = bfaces.empty() ? nullptr : bfaces.data();
  d.bface_kind = bkind.empty() ? nullptr : bkind.data();
  d.part = part.empty() ? nullptr : part.data();
  d.n_sub = n_sub;
  d.overlap_layers = overlap;
  d.k0 = k0;
  d.degree = degree;
  d.precision = precision;
  d.prec_variant = variant;

  mxw::Layout L;
  const mxw_status st = mxw::build_layout(&d, L);
  {
    std::ofstream s(dir + "/status.txt");
    s << (int)st << "\n" << (st == MXW_OK ? std::string("ok") : mxw::g_error) << "\n";
  }
  if (st != MXW_OK) return 0;

  {
    std::ofstream s(dir + "/info.txt");
    s << L.ndof << " " << L.cols.size() << " " << L.n_sub << " " << L.sum_ns << " " << L.max_ns << " "
      << L.n_iface << " " << L.basis.nloc << "\n";
  }
  save(dir + "/rowptr.bin", L.rowptr);
  save(dir + "/cols.bin", L.cols);
  save(dir + "/ent_kind.bin", L.ent_kind);
  save(dir + "/ent_id.bin", L.ent_id);
  save(dir + "/ent_local.bin", L.ent_local);
  save(dir + "/sub_ptr.bin", L.sub_dof_ptr);
  save(dir + "/sub_dofs.bin", L.sub_dofs);
  save(dir + "/sub_pou.bin", L.sub_pou);
  save(dir + "/imp_tet.bin", L.imp_tet);
  save(dir + "/sub_face_tet.bin", L.sub_face_tet);

  std::vector<double> imp_beta, sub_face_coef;
  mxw::face_coefficients(L, L.eps.data(), L.k0, imp_beta, sub_face_coef);
  save(dir + "/imp_beta.bin", imp_beta);
  save(dir + "/sub_face_coef.bin", sub_face_coef);
  return 0;
}
