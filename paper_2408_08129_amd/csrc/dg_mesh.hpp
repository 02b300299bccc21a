// Host mesh description produced by build_mesh (see dg_mesh.cpp).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/imexdg.h"

namespace dg {

enum HostFaceKind : int { kWall = 0, kConf = 1, kFine = 2, kCoarse = 3 };

struct HostMesh {
  int dim = 0, degree = 0, np = 0, nloc = 0;
  int nb[3] = {1, 1, 1};     // base cells per axis (3D x,y,z; 2D x,z)
  double L[3] = {1, 1, 1};   // extents per axis
  int per[3] = {0, 0, 0};
  int lmax = 0;
  int ncell = 0;
  long nhang = 0;            // hanging sub-faces, each counted once (on the coarse side)
  std::vector<int> cell;     // 4 per cell: level, i0, i1, i2
  std::vector<int> fkind;    // 2 d per cell
  std::vector<int> fnbr;     // 4 per face
};

int build_mesh(const dg_case_desc& cs, int degree, HostMesh& M, std::string& err);

}  // namespace dg
