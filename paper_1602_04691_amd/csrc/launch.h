// Kernel launches of the library (host side).
//
// Every launch goes through launch_kernel.  Normally it launches on the
// stream.  While the calling thread builds a HIP graph of COCG iterations
// (graph_being_built() not NULL), the same call appends a kernel node with
// the same grid, block and arguments after the graph's previous node
// instead: the graph is assembled node by node, and no stream is ever put
// into capture mode, so HIP calls that other threads make at the same time
// (their own launches, allocations, copies) cannot interfere with it.
#pragma once

#include <hip/hip_runtime.h>

#include <tuple>
#include <type_traits>
#include <utility>

namespace ori {

struct GraphBuild {
  hipGraph_t graph = nullptr;
  hipGraphNode_t last = nullptr;  // the node the next one depends on (NULL: none yet)
};

// The graph the calling thread is building, or NULL (thread local; defined
// in the host runtime).
GraphBuild* graph_being_built();

template <class... P, class... A, size_t... I>
hipError_t launch_kernel_impl(void (*k)(P...), dim3 grid, dim3 block, unsigned smem, hipStream_t st,
                              std::index_sequence<I...>, A&&... args) {
  // the arguments converted to the kernel's parameter types, one address each
  std::tuple<std::decay_t<P>...> vals(std::forward<A>(args)...);
  void* params[sizeof...(P) + 1] = {static_cast<void*>(&std::get<I>(vals))..., nullptr};
  if (GraphBuild* gb = graph_being_built()) {
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(k);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = smem;
    kp.kernelParams = params;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e =
        hipGraphAddKernelNode(&node, gb->graph, gb->last ? &gb->last : nullptr, gb->last ? 1 : 0, &kp);
    if (e == hipSuccess) gb->last = node;
    return e;
  }
  return hipLaunchKernel(reinterpret_cast<const void*>(k), grid, block, params, smem, st);
}

// k<<<grid, block, 0, st>>>(args...), or a node of the graph being built.
template <class... P, class... A>
hipError_t launch_kernel(void (*k)(P...), dim3 grid, dim3 block, hipStream_t st, A&&... args) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  return launch_kernel_impl(k, grid, block, 0u, st, std::index_sequence_for<P...>{}, std::forward<A>(args)...);
}

// The same with smem bytes of dynamic LDS.
template <class... P, class... A>
hipError_t launch_kernel_smem(void (*k)(P...), dim3 grid, dim3 block, unsigned smem, hipStream_t st, A&&... args) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  return launch_kernel_impl(k, grid, block, smem, st, std::index_sequence_for<P...>{}, std::forward<A>(args)...);
}

}  // namespace ori
