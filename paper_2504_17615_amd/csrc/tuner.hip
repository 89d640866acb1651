// Degree-class cut-off tables and the cache of the autotuner.
#include "tuner.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <stdexcept>

namespace lmgp {

ClassCuts default_cuts() {
  return ClassCuts{{4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 6144, 8192}};
}

// Dense rows: one wave per node up to degree 512, a 256-thread block per node
// up to 8192 (classes 10 and 11, the 1024-thread rows, stay empty), hub rows
// above.
ClassCuts dense_cuts() {
  return ClassCuts{{4, 8, 16, 32, 64, 128, 256, 512, 1024, 8192, 8192, 8192}};
}

const std::vector<CutPreset>& cut_presets(bool dense) {
  // hashed tables: lane groups hold degree <= 2G (two entries per lane) or
  // <= G (one); block tables run at load <= 1/2 or <= 3/4; the largest LDS
  // table may take degrees up to 12288 before the global-table path
  static const std::vector<CutPreset> hashed = {
      {"default", default_cuts()},
      {"lanes1", {{2, 4, 8, 16, 32, 64, 256, 512, 1024, 2048, 6144, 8192}}},
      {"load34", {{4, 8, 16, 32, 64, 128, 384, 768, 1536, 3072, 6144, 12288}}},
      {"lanes1+load34", {{2, 4, 8, 16, 32, 64, 384, 768, 1536, 3072, 6144, 12288}}},
      {"big3072", {{4, 8, 16, 32, 64, 128, 256, 512, 1024, 3072, 6144, 8192}}},
  };
  // dense rows (refinement, few blocks): the bounds that matter are the end
  // of the lane groups (class 5), of the one-wave rows (class 7), of the
  // 256-thread rows (class 9) and of the 1024-thread rows (class 11)
  static const std::vector<CutPreset> rows = {
      {"default", dense_cuts()},
      {"rows256", {{4, 8, 16, 32, 64, 128, 128, 128, 1024, 2048, 6144, 8192}}},
      {"waves2048", {{4, 8, 16, 32, 64, 128, 1024, 2048, 2048, 2048, 6144, 8192}}},
      {"rows1024", {{4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 6144, 8192}}},
      {"waves1024", {{4, 8, 16, 32, 64, 128, 512, 1024, 1024, 8192, 8192, 8192}}},
      {"waves8192", {{4, 8, 16, 32, 64, 128, 4096, 8192, 8192, 8192, 8192, 8192}}},
      {"groups64", {{4, 8, 16, 32, 64, 64, 256, 512, 1024, 8192, 8192, 8192}}},
      {"wide32768", {{4, 8, 16, 32, 64, 128, 256, 512, 1024, 8192, 8192, 32768}}},
  };
  static const bool checked = [] {
    for (const CutPreset& p : hashed)
      if (!cuts_valid(p.cuts, false)) throw std::logic_error(std::string("bad table ") + p.name);
    for (const CutPreset& p : rows)
      if (!cuts_valid(p.cuts, true)) throw std::logic_error(std::string("bad table ") + p.name);
    return true;
  }();
  (void)checked;
  return dense ? rows : hashed;
}

bool cuts_valid(const ClassCuts& c, bool dense) {
  for (int i = 1; i < NCLASS - 1; ++i)
    if (c.ub[i] < c.ub[i - 1]) return false;
  // lane group of G lanes: two entries per lane, degree <= 2G
  for (int i = 0; i < CLASS_BLOCK; ++i)
    if (c.ub[i] > (4u << i)) return false;
  if (dense) return true;  // per-block rows hold any degree
  // hashed LDS tables: at most 3/4 of the slots used
  for (int i = CLASS_BLOCK; i < CLASS_GLOBAL; ++i)
    if ((uint64_t)c.ub[i] * 4 > 3ull << class_table_log(i)) return false;
  return true;
}

std::string tune_key(int phase, bool dense, int ew_kind, bool packed,
                     const uint64_t* class_count) {
  std::ostringstream o;
  o << (phase ? "rf" : "cl") << (dense ? "/rows" : "/hash") << "/e" << ew_kind
    << (packed ? "/p" : "/u") << ':';
  for (int c = 0; c < NCLASS; ++c) {
    int bits = 0;
    for (uint64_t v = class_count[c]; v; v >>= 1) ++bits;
    o << (char)(bits < 10 ? '0' + bits : 'a' + bits - 10);
  }
  return o.str();
}

Tuner& Tuner::get() {
  static Tuner t;
  return t;
}

void Tuner::load_locked() {
  if (loaded_) return;
  loaded_ = true;
  const char* path = std::getenv("LMGP_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string key;
  int preset;
  while (f >> key >> preset) cache_[key] = preset;
}

int Tuner::lookup(const std::string& key) {
  std::lock_guard<std::mutex> g(mu_);
  load_locked();
  auto it = cache_.find(key);
  return it == cache_.end() ? -1 : it->second;
}

void Tuner::store(const std::string& key, int preset) {
  std::lock_guard<std::mutex> g(mu_);
  load_locked();
  cache_[key] = preset;
  const char* path = std::getenv("LMGP_TUNE_CACHE");
  if (path && *path) {
    std::ofstream f(path, std::ios::app);
    f << key << ' ' << preset << '\n';
  }
}

void Tuner::note_trial() {
  std::lock_guard<std::mutex> g(mu_);
  ++trials_;
}

uint64_t Tuner::entries() {
  std::lock_guard<std::mutex> g(mu_);
  return cache_.size();
}

uint64_t Tuner::trials() {
  std::lock_guard<std::mutex> g(mu_);
  return trials_;
}

void Tuner::clear() {
  std::lock_guard<std::mutex> g(mu_);
  cache_.clear();
  trials_ = 0;
  loaded_ = true;  // do not re-read the file after an explicit clear
}

}  // namespace lmgp
