// Work ring of the served path: the host scheduler publishes work items into
// pinned host memory and one persistent kernel (k_served) claims them while
// it runs, so that a request reaches the compute units without a kernel
// launch of its own.
//
// Items.  A solve is published as one prep item, into the prep queue, and
// one tile item per tile, into the tile queue:
//  - prep: copy the solve's upload block (descriptor + request data, `count`
//    bytes) from its pinned mirror `src` into its device block (at offset
//    `block` of the pool, so that the kernel addresses it as global memory
//    derived from its own argument), fold the latent block of every gate
//    (FP64), then mark the slot's block ready with the solve's sequence
//    number;
//  - tile (k0 >= 0): wait until the slot's block is ready, run the tile of 16
//    rollouts starting at k0 (noise, dynamics, decoder, costs, tile partial),
//    and count it; the workgroup that counts the solve's last tile merges the
//    tile partials (FP64, fixed order) and writes the result, the warm start
//    and the tick, then publishes the solve's sequence number in the slot's
//    completion word;
//  - exit (k0 = kRingExit, tile queue only): the workgroup leaves.
// A workgroup looking for work takes a prep item whenever one is queued
// (compare-and-swap on the prep head; preps are few), and otherwise the item
// of its ticket: a tile-queue index taken by fetch-and-add, so that claims
// never contend, held until the host has published that index.  A tile whose
// block is not ready yet takes and runs queued prep items itself while it
// waits; prep items wait on nothing, so every wait of a tile ends.  The host
// rewrites an item only once its solve has completed, which cannot happen
// before the item was read.
//
// Memory.  items, pitems, tail, ptail, done and lost live in pinned host
// memory (coherent; the device reads host words with relaxed system-scope
// loads and writes done after a system-scope release); head, phead, prep,
// tiles, fail and the device copies of the tails live in device memory.
// Workgroups look for work in the device copies only: one workgroup at a
// time (a token), at most once per `refresh_ticks` of the real-time clock,
// reads the host tails and raises the copies, so the polling of host memory
// over the bus does not grow with the grid.  Polling never fences (a fence
// at agent or system scope writes back or invalidates a whole L2 here).
// Results, normalised weights and a copy of the costs go straight to pinned
// per-slot areas named in the descriptor.
//
// Exit.  The host ends a launch by publishing one exit item per workgroup
// into the tile queue (after a quiet period, or at destroy): every workgroup
// holds at most one ticket and takes exactly one exit, so every ticket is
// filled and nothing is left half-claimed; items published after the exits
// wait for the next launch.  Bounded waits end every wave even without the
// host: a ticket not published within `wait_polls` polls makes its workgroup
// leave and set `lost` (the host then treats the device as failed), and a
// tile gives up waiting for its block after `wait_polls` polls and marks the
// slot failed (the solve completes with an error).
#pragma once
#include <stdint.h>

namespace mppi {

struct RingItem {
  uint64_t block;   // byte offset of the solve's block (descriptor first) in the device pool
  uint64_t src;     // prep: device-visible address of the pinned upload mirror
  uint32_t slot;    // solve slot (counters, completion word)
  int32_t k0;       // tile: first rollout; prep: -1; exit: kRingExit
  uint32_t count;   // prep: upload bytes (multiple of 16); tile: the solve's tile count
  uint32_t seq;     // the solve's sequence number (1 .. 2^31 - 1)
};
static_assert(sizeof(RingItem) == 32, "ring items are 32 bytes");

constexpr int32_t kRingExit = -2;

// Completion word of a slot: the solve's sequence number, with this bit set
// when a tile gave up waiting for its block (the solve failed).
constexpr uint32_t kRingFailBit = 0x80000000u;

struct RingArgs {
  char* pool;              // device pool holding the solves' blocks
  const RingItem* items;   // pinned: tile queue, cap items, item i at i % cap
  const RingItem* pitems;  // pinned: prep queue, pcap items
  const uint64_t* tail;    // pinned: tile items published
  const uint64_t* ptail;   // pinned: prep items published
  uint32_t* done;          // pinned: per slot, completion word
  uint32_t* lost;          // pinned: set when a workgroup left with an unfilled ticket
  uint64_t* head;          // device: tickets taken
  uint64_t* phead;         // device: prep items claimed
  uint32_t* prep;          // device: per slot, sequence number whose block is ready
  uint32_t* tiles;         // device: per slot, tiles counted
  uint32_t* fail;          // device: per slot, a tile gave up waiting
  uint64_t* dtail;         // device copies of tail and ptail
  uint64_t* dptail;
  uint32_t* poll;          // device: token of the workgroup reading the host tails
  uint64_t* poll_time;     // device: real-time clock of the last read
  uint32_t cap, pcap;
  uint32_t wait_polls;
  uint32_t refresh_ticks;  // real-time clock ticks (100 MHz) between reads of the host tails
};

}  // namespace mppi
