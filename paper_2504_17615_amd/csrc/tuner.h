// Autotuning of the rating kernels' degree classes.
//
// The rating pass sends every active node to a kernel chosen by its degree
// (lane groups, one block, one 1024-thread block, global tables).  Where the
// cut-offs between those kernels pay off depends on the degree histogram of
// the level and on the phase, so a small set of cut-off tables is kept, each
// of which routes every degree to a kernel able to hold it: the choice moves
// work between kernels and never changes a result.  The tuner times each
// table on the first sub-round of a level whose (phase, table kind, degree
// histogram) it has not seen and caches the fastest; later levels and calls
// with the same signature reuse it.  The cache lives for the process and, if
// LMGP_TUNE_CACHE names a file, is read from and appended to that file.
#pragma once
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

namespace lmgp {

// Levels whose rating pass reads fewer CSR entries keep the default table:
// their launches are too short to time reliably and gain little.
constexpr uint64_t TUNE_MIN_ENTRIES = 1ull << 21;

struct CutPreset {
  const char* name;
  ClassCuts cuts;
};

// The table of degree_class (preset 0 of both kinds).
ClassCuts default_cuts();
// The default table of refinement with dense per-block rows.
ClassCuts dense_cuts();
// Tables for the hashed rating kernels (dense = false) and for refinement
// with dense per-block rows (dense = true).
const std::vector<CutPreset>& cut_presets(bool dense);
// Whether every class of `c` holds the degrees it is given.
bool cuts_valid(const ClassCuts& c, bool dense);
// Cache key: phase, kind, weight width, packing and the per-class node
// counts of the level (as bit lengths, a log-scale degree histogram).
std::string tune_key(int phase, bool dense, int ew_kind, bool packed,
                     const uint64_t* class_count);

class Tuner {
 public:
  static Tuner& get();
  int lookup(const std::string& key);  // cached preset, or -1
  void store(const std::string& key, int preset);
  void note_trial();
  uint64_t entries();
  uint64_t trials();
  void clear();  // forget the process cache (the file is left as it is)

 private:
  void load_locked();
  std::mutex mu_;
  std::map<std::string, int> cache_;
  bool loaded_ = false;
  uint64_t trials_ = 0;
};

}  // namespace lmgp
