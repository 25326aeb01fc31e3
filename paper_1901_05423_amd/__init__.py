"""MI355X-native radix tree forests for monotone inverse-CDF sampling."""
