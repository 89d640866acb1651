// Initial partitioning on the device: the recursive bisection by greedy
// graph growing that the host version (initial_partition_host) computes,
// with the subproblems of one recursion depth bisected concurrently, one
// workgroup each.
#pragma once
#include <vector>

#include "common.h"
#include "memory.h"

namespace lmgp {

constexpr uint32_t IP_NONE = 0xFFFFFFFFu;

// One subproblem: a node set receiving the kS blocks starting at its global
// block id; part 1 gets the first k1 = ceil(kS / 2) of them.
struct IpSub {
  uint64_t pre;  // H(seed, IP, level, off, kS): start order of the node set
  uint64_t n0;   // first node of its graph (hashes take graph-local ids)
  uint32_t kS, k1;
};

// A level (union of graphs) whose graphs are partitioned; part[b] = 1 for
// the graphs taking part (their coarsest level is this one).
struct IpLevel {
  const uint64_t* xadj;
  const uint32_t* adj;
  const int64_t* nw;
  const uint32_t* gid;  // NULL for a single graph
  uint64_t n;
};

class IpDevice {
 public:
  // boff: block id of every node of the taking-part graphs (their first
  // global block on entry); updated in place depth by depth.
  IpDevice(const IpLevel& L, uint32_t* boff, uint64_t nblocks, Pool& pool, hipStream_t s);
  // One depth: subs[i] is subproblem i; sub_of_block[K] = the subproblem whose
  // node set holds the nodes now in block K (IP_NONE: finished).
  void depth(const std::vector<IpSub>& subs, const std::vector<uint32_t>& sub_of_block);
  // Throws if a workgroup hit its iteration guard (a bug, never expected).
  void finish();

 private:
  IpLevel L_;
  uint32_t* boff_;
  uint64_t nblocks_;
  Pool& pool_;
  hipStream_t s_;
  DBuf<uint32_t> sub_, queue_, jl_, err_;
  DBuf<uint64_t> dpre_, keys_, keys2_;
  DBuf<uint32_t> vals_, vals2_;
  DBuf<uint8_t> visited_, part1_;
  DBuf<unsigned long long> first_;
  // host tables of the depths in flight (their copies may still be running)
  std::vector<std::vector<IpSub>> hold_subs_;
  std::vector<std::vector<uint32_t>> hold_sob_;
};

// boff[v] = gbase[graph of v] (IP_NONE for graphs that do not take part).
void ip_device_init(const uint32_t* gid, const uint32_t* gbase_dev, uint64_t n, uint32_t* boff,
                    hipStream_t s);

}  // namespace lmgp
